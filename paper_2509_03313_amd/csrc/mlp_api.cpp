// mlp_api.cpp -- C ABI of the inter-pulse surrogate perceptron (include/gsbs.h,
// gsbs_mlp_*): device buffers, forward pass, backward pass, Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"
#include "gsbs.h"
#include "mlp.h"

using namespace gsbs;

namespace {

#define MHIP(x)                                                                                         \
    do {                                                                                                \
        hipError_t e_ = (x);                                                                            \
        if (e_ != hipSuccess) return set_error(GSBS_EHIP, (std::string(#x) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

// every matrix dimension of the products is a multiple of 32 (the K step of the MFMA)
constexpr int pad32(int v) { return (v + 31) / 32 * 32; }

// Padded layer shapes: K inputs (valid kv), N outputs (valid nv).
struct Shape {
    int K, N, kv, nv;
};
constexpr Shape kShape[kMlpLayers] = {{pad32(kMlpIn), kMlpHidden, kMlpIn, kMlpHidden},
                                      {kMlpHidden, kMlpHidden, kMlpHidden, kMlpHidden},
                                      {kMlpHidden, kMlpHidden, kMlpHidden, kMlpHidden},
                                      {kMlpHidden, kMlpHidden, kMlpHidden, kMlpHidden},
                                      {kMlpHidden, pad32(kMlpOut), kMlpHidden, kMlpOut}};

template <typename T>
int zalloc(T** p, size_t n, hipStream_t st) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, n * sizeof(T));
    if (e != hipSuccess) return set_error(GSBS_ENOMEM, (std::string("hipMalloc: ") + hipGetErrorString(e)).c_str());
    e = hipMemsetAsync(q, 0, n * sizeof(T), st);
    if (e != hipSuccess) return set_error(GSBS_EHIP, hipGetErrorString(e));
    *p = (T*)q;
    return GSBS_OK;
}

#define MCHK(x)                       \
    do {                              \
        int r_ = (x);                 \
        if (r_ != GSBS_OK) return r_; \
    } while (0)

int64_t n_params() {
    int64_t n = 0;
    for (const Shape& s : kShape) n += (int64_t)s.nv * s.kv + s.nv;
    return n;
}

}  // namespace

struct gsbs_mlp {
    hipStream_t st = nullptr;
    int max_batch = 0, Mp_max = 0;
    int64_t step = 0;
    // per layer: FP32 master weights [N][K] and biases, Adam moments, gradients, BF16 copies
    float *w[kMlpLayers] = {}, *m1[kMlpLayers] = {}, *m2[kMlpLayers] = {}, *gw[kMlpLayers] = {};
    float *b[kMlpLayers] = {}, *bm1[kMlpLayers] = {}, *bm2[kMlpLayers] = {}, *gb[kMlpLayers] = {};
    uint16_t *wb[kMlpLayers] = {}, *wbt[kMlpLayers] = {};
    // activations entering layer l (BF16 and transpose), hidden pre-activations
    uint16_t *act[kMlpLayers] = {}, *actT[kMlpLayers] = {};
    float* Z[kMlpLayers] = {};
    float *Y = nullptr, *dZ = nullptr, *dA = nullptr, *loss = nullptr;
    // partial products of split reductions (weight gradients, bias gradients)
    float* work = nullptr;
    size_t work_elems = 0;
    uint16_t *dZb = nullptr, *dZT = nullptr;
    std::vector<void*> owned;
};

namespace {

template <typename T>
int own(gsbs_mlp* m, T** p, size_t n) {
    MCHK(zalloc(p, n, m->st));
    m->owned.push_back((void*)*p);
    return GSBS_OK;
}

// Flat FP32 layout of the ABI: per layer W[nv][kv] row-major, then b[nv].
int copy_params(gsbs_mlp* m, float* const* dev_w, float* const* dev_b, const float* host, float* out_host) {
    int64_t off = 0;
    for (int l = 0; l < kMlpLayers; ++l) {
        const Shape& s = kShape[l];
        std::vector<float> pw((size_t)s.N * s.K, 0.0f), pb((size_t)s.N, 0.0f);
        if (host) {
            for (int n = 0; n < s.nv; ++n)
                for (int k = 0; k < s.kv; ++k) pw[(size_t)n * s.K + k] = host[off + (int64_t)n * s.kv + k];
            off += (int64_t)s.nv * s.kv;
            for (int n = 0; n < s.nv; ++n) pb[n] = host[off + n];
            off += s.nv;
            MHIP(hipMemcpyAsync(dev_w[l], pw.data(), pw.size() * 4, hipMemcpyHostToDevice, m->st));
            MHIP(hipMemcpyAsync(dev_b[l], pb.data(), pb.size() * 4, hipMemcpyHostToDevice, m->st));
            MHIP(hipStreamSynchronize(m->st));
        } else {
            MHIP(hipMemcpyAsync(pw.data(), dev_w[l], pw.size() * 4, hipMemcpyDeviceToHost, m->st));
            MHIP(hipMemcpyAsync(pb.data(), dev_b[l], pb.size() * 4, hipMemcpyDeviceToHost, m->st));
            MHIP(hipStreamSynchronize(m->st));
            for (int n = 0; n < s.nv; ++n)
                for (int k = 0; k < s.kv; ++k) out_host[off + (int64_t)n * s.kv + k] = pw[(size_t)n * s.K + k];
            off += (int64_t)s.nv * s.kv;
            for (int n = 0; n < s.nv; ++n) out_host[off + n] = pb[n];
            off += s.nv;
        }
    }
    return GSBS_OK;
}

// train: also keep what the backward pass reads (pre-activations, transposed
// activations).
int forward(gsbs_mlp* m, const float* x, int B, float* y, bool train) {
    const int Mp = pad32(B);
    mlp_input(m->st, x, B, kMlpIn, m->act[0], train ? m->actT[0] : nullptr, Mp, kShape[0].K);
    for (int l = 0; l < kMlpLayers; ++l) {
        const Shape& s = kShape[l];
        const bool hidden = l + 1 < kMlpLayers;
        mlp_gemm_layer(m->st, m->act[l], m->wb[l], Mp, s.N, s.K, m->b[l], B, s.nv, hidden ? 1 : 0,
                       train ? m->Z[l] : nullptr, hidden ? m->act[l + 1] : nullptr,
                       (hidden && train) ? m->actT[l + 1] : nullptr, y);
    }
    MHIP(hipGetLastError());
    return GSBS_OK;
}

int check(gsbs_mlp* m, const void* x, int32_t B) {
    if (!m || !x) return set_error(GSBS_EINVAL, "null");
    if (B < 1 || B > m->max_batch) return set_error(GSBS_EINVAL, "batch outside 1..max_batch");
    return GSBS_OK;
}

}  // namespace

extern "C" {

int gsbs_mlp_param_count(int64_t* n) {
    if (!n) return set_error(GSBS_EINVAL, "null");
    *n = n_params();
    return GSBS_OK;
}

int gsbs_mlp_create(int32_t max_batch, void* stream, gsbs_mlp** out) {
    if (!out || max_batch < 1 || max_batch > (1 << 20)) return set_error(GSBS_EINVAL, "bad arguments");
    gsbs_mlp* m = new gsbs_mlp();
    m->st = (hipStream_t)stream;
    m->max_batch = max_batch;
    m->Mp_max = pad32(max_batch);
    const int Mp = m->Mp_max;
    int r = GSBS_OK;
    for (int l = 0; l < kMlpLayers && r == GSBS_OK; ++l) {
        const Shape& s = kShape[l];
        const size_t nw = (size_t)s.N * s.K;
        if ((r = own(m, &m->w[l], nw)) || (r = own(m, &m->m1[l], nw)) || (r = own(m, &m->m2[l], nw)) ||
            (r = own(m, &m->gw[l], nw)) || (r = own(m, &m->b[l], (size_t)s.N)) || (r = own(m, &m->bm1[l], (size_t)s.N)) ||
            (r = own(m, &m->bm2[l], (size_t)s.N)) || (r = own(m, &m->gb[l], (size_t)s.N)) ||
            (r = own(m, &m->wb[l], nw)) || (r = own(m, &m->wbt[l], nw)) ||
            (r = own(m, &m->act[l], (size_t)Mp * s.K)) || (r = own(m, &m->actT[l], (size_t)Mp * s.K)) ||
            (r = own(m, &m->Z[l], (size_t)Mp * s.N)))
            break;
    }
    const size_t wide = (size_t)Mp * kShape[0].K;
    if (r == GSBS_OK &&
        ((r = own(m, &m->Y, (size_t)Mp * kMlpOut)) || (r = own(m, &m->dZ, wide)) ||
         (r = own(m, &m->dA, wide)) || (r = own(m, &m->loss, 1)) || (r = own(m, &m->dZb, wide)) ||
         (r = own(m, &m->dZT, wide)))) {
    }
    // split reductions: at most 64 slices (and Mp / 512) of the largest weight
    // gradient, and the column-sum chunks
    const size_t slices = std::min<size_t>(64, (size_t)Mp / 512 + 1);
    m->work_elems = std::max(slices * (size_t)kMlpHidden * kShape[0].K, ((size_t)Mp / 512 + 1) * kShape[0].K);
    if (r == GSBS_OK) r = own(m, &m->work, m->work_elems);
    if (r == GSBS_OK && hipStreamSynchronize(m->st) != hipSuccess) r = set_error(GSBS_EHIP, "stream");
    if (r != GSBS_OK) {
        for (void* p : m->owned) (void)hipFree(p);
        delete m;
        return r;
    }
    *out = m;
    return GSBS_OK;
}

int gsbs_mlp_destroy(gsbs_mlp* m) {
    if (!m) return GSBS_OK;
    (void)hipStreamSynchronize(m->st);
    for (void* p : m->owned) (void)hipFree(p);
    delete m;
    return GSBS_OK;
}

int gsbs_mlp_set_weights(gsbs_mlp* m, const float* w, int64_t n) {
    if (!m || !w) return set_error(GSBS_EINVAL, "null");
    if (n != n_params()) return set_error(GSBS_EINVAL, "parameter count differs from gsbs_mlp_param_count");
    MCHK(copy_params(m, m->w, m->b, w, nullptr));
    for (int l = 0; l < kMlpLayers; ++l) {
        const Shape& s = kShape[l];
        const size_t nw = (size_t)s.N * s.K;
        MHIP(hipMemsetAsync(m->m1[l], 0, nw * 4, m->st));
        MHIP(hipMemsetAsync(m->m2[l], 0, nw * 4, m->st));
        MHIP(hipMemsetAsync(m->bm1[l], 0, (size_t)s.N * 4, m->st));
        MHIP(hipMemsetAsync(m->bm2[l], 0, (size_t)s.N * 4, m->st));
        mlp_cast(m->st, m->w[l], (int64_t)nw, s.N, s.K, m->wb[l], m->wbt[l]);
    }
    m->step = 0;
    MHIP(hipGetLastError());
    MHIP(hipStreamSynchronize(m->st));
    return GSBS_OK;
}

int gsbs_mlp_get_weights(gsbs_mlp* m, float* w, int64_t n) {
    if (!m || !w) return set_error(GSBS_EINVAL, "null");
    if (n != n_params()) return set_error(GSBS_EINVAL, "parameter count differs from gsbs_mlp_param_count");
    return copy_params(m, m->w, m->b, nullptr, w);
}

int gsbs_mlp_get_grads(gsbs_mlp* m, float* g, int64_t n) {
    if (!m || !g) return set_error(GSBS_EINVAL, "null");
    if (n != n_params()) return set_error(GSBS_EINVAL, "parameter count differs from gsbs_mlp_param_count");
    return copy_params(m, m->gw, m->gb, nullptr, g);
}

int gsbs_mlp_forward(gsbs_mlp* m, const float* x, int32_t batch, float* y) {
    MCHK(check(m, x, batch));
    if (!y) return set_error(GSBS_EINVAL, "null");
    return forward(m, x, batch, y, false);
}

// Forward pass for the surrogate hand-over of gsbs_advance_to: x, y device
// arrays; returns once y is written.
extern "C++" int gsbs::mlp_forward_sync(gsbs_mlp* m, const float* x, int batch, float* y) {
    MCHK(gsbs_mlp_forward(m, x, batch, y));
    MHIP(hipStreamSynchronize(m->st));
    return GSBS_OK;
}

int gsbs_mlp_get_activation(gsbs_mlp* m, int32_t layer, int32_t batch, float* out) {
    if (!m || !out) return set_error(GSBS_EINVAL, "null");
    if (layer < 0 || layer >= kMlpLayers || batch < 1 || batch > m->max_batch)
        return set_error(GSBS_EINVAL, "layer or batch out of range");
    const Shape& s = kShape[layer];
    std::vector<uint16_t> h((size_t)pad32(batch) * s.K);
    MHIP(hipMemcpyAsync(h.data(), m->act[layer], h.size() * 2, hipMemcpyDeviceToHost, m->st));
    MHIP(hipStreamSynchronize(m->st));
    for (int r = 0; r < batch; ++r)
        for (int k = 0; k < s.kv; ++k) {
            const uint32_t u = (uint32_t)h[(size_t)r * s.K + k] << 16;
            float f;
            std::memcpy(&f, &u, 4);
            out[(size_t)r * s.kv + k] = f;
        }
    return GSBS_OK;
}

int gsbs_mlp_backward(gsbs_mlp* m, const float* x, const float* t, int32_t batch, float* loss) {
    MCHK(check(m, x, batch));
    if (!t) return set_error(GSBS_EINVAL, "null");
    const int B = batch, Mp = pad32(batch);
    MCHK(forward(m, x, B, m->Y, true));
    MHIP(hipMemsetAsync(m->loss, 0, 4, m->st));
    const Shape& so = kShape[kMlpLayers - 1];
    mlp_loss(m->st, m->Y, t, B, kMlpOut, Mp, so.N, m->dZ, m->dZb, m->dZT, m->loss);
    for (int l = kMlpLayers - 1; l >= 0; --l) {
        const Shape& s = kShape[l];
        // dW = dZ^T X, db = column sums of dZ
        mlp_gemm_nt(m->st, m->dZT, Mp, m->actT[l], Mp, m->gw[l], s.K, s.N, s.K, Mp, m->work, m->work_elems);
        mlp_colsum(m->st, m->dZ, Mp, s.N, m->gb[l], m->work);
        if (l == 0) break;
        // dA = dZ W, then dZ of the layer below through GELU'
        mlp_gemm_nt(m->st, m->dZb, s.N, m->wbt[l], s.N, m->dA, s.K, Mp, s.K, s.N, nullptr, 0);
        mlp_act_grad(m->st, m->dA, m->Z[l - 1], B, Mp, s.K, kShape[l - 1].nv, m->dZ, m->dZb, m->dZT);
    }
    MHIP(hipGetLastError());
    if (loss) {
        float h = 0.f;
        MHIP(hipMemcpyAsync(&h, m->loss, 4, hipMemcpyDeviceToHost, m->st));
        MHIP(hipStreamSynchronize(m->st));
        *loss = h / (float)(B * kMlpOut);
    }
    return GSBS_OK;
}

int gsbs_mlp_adam(gsbs_mlp* m, float lr, float beta1, float beta2, float eps) {
    if (!m) return set_error(GSBS_EINVAL, "null");
    if (!(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return set_error(GSBS_EINVAL, "bad Adam parameters");
    m->step += 1;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)m->step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)m->step));
    for (int l = 0; l < kMlpLayers; ++l) {
        const Shape& s = kShape[l];
        mlp_adam(m->st, m->w[l], m->m1[l], m->m2[l], m->gw[l], (int64_t)s.N * s.K, s.N, s.K, lr, beta1, beta2, eps, c1,
                 c2, m->wb[l], m->wbt[l]);
        mlp_adam(m->st, m->b[l], m->bm1[l], m->bm2[l], m->gb[l], s.N, 1, s.N, lr, beta1, beta2, eps, c1, c2, nullptr,
                 nullptr);
    }
    MHIP(hipGetLastError());
    return GSBS_OK;
}

int gsbs_mlp_train_step(gsbs_mlp* m, const float* x, const float* t, int32_t batch, float lr, float beta1,
                        float beta2, float eps, float* loss) {
    MCHK(gsbs_mlp_backward(m, x, t, batch, loss));
    return gsbs_mlp_adam(m, lr, beta1, beta2, eps);
}

}  // extern "C"

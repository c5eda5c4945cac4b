// Host side of the proposal network: the C ABI of include/prop.h.
#include "prop.h"
#include "prop_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <random>
#include <string>
#include <vector>

namespace {

thread_local std::string g_error = "no error";

struct PropError {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw PropError{code, buf};
}

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? CORR_ENOMEM : CORR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// parameter layout (floats)
constexpr int64_t kW1 = 0, kB1 = kW1 + 160 * 256, kW2 = kB1 + 256, kB2 = kW2 + 256 * 256, kW3 = kB2 + 256,
                  kB3 = kW3 + 256 * 256, kW4 = kB3 + 256, kB4 = kW4 + 256, kNP = kB4 + 1;
static_assert(kNP == PROP_NPARAMS, "parameter count");

template <class T>
T* dalloc(std::vector<void*>& owned, size_t count) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(T) * std::max<size_t>(count, 1));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(CORR_ENOMEM, "hipMalloc(%zu): %s", sizeof(T) * count, hipGetErrorString(e));
    }
    owned.push_back(p);
    return static_cast<T*>(p);
}

}  // namespace

struct prop_ctx {
    hipStream_t stream = nullptr;
    int batch = 0;
    uint64_t seed = 0;
    int64_t step = 0;  // Adam steps taken
    std::vector<void*> owned;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // [kNP]
    uint16_t* pb = nullptr;                                         // bf16 copy [kNP]
    uint16_t* xb = nullptr;                                         // [batch][160]
    float* yb = nullptr;                                            // [batch] targets
    float* y = nullptr;                                             // [batch] outputs
    float *z1 = nullptr, *z2 = nullptr, *z3 = nullptr;              // [batch][256]
    uint16_t *a1 = nullptr, *a2 = nullptr, *a3 = nullptr;           // [batch][256]
    uint16_t *d1 = nullptr, *d2 = nullptr, *d3 = nullptr;           // [batch][256] gradients at z
    float* loss = nullptr;                                          // [1]
    std::string err = "no error";
};

namespace {

template <class F>
int guarded(prop_ctx* c, F&& body) {
    try {
        body();
        return CORR_OK;
    } catch (const PropError& e) {
        (c ? c->err : g_error) = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        (c ? c->err : g_error) = "host allocation failed";
        return CORR_ENOMEM;
    } catch (...) {
        (c ? c->err : g_error) = "unexpected internal error";
        return CORR_EHIP;
    }
}

void forward(prop_ctx* c, int rows) {
    using namespace prop;
    hipStream_t st = c->stream;
    Epi_args e;
    e.mode = kEpiHidden;
    e.bias = c->p + kB1; e.z = c->z1; e.act = c->a1;
    hip_check(gemm(false, false, c->xb, kIn, c->pb + kW1, kHidden, rows, kHidden, kIn, e, st), "gemm 1");
    e.bias = c->p + kB2; e.z = c->z2; e.act = c->a2;
    hip_check(gemm(false, false, c->a1, kHidden, c->pb + kW2, kHidden, rows, kHidden, kHidden, e, st), "gemm 2");
    e.bias = c->p + kB3; e.z = c->z3; e.act = c->a3;
    hip_check(gemm(false, false, c->a2, kHidden, c->pb + kW3, kHidden, rows, kHidden, kHidden, e, st), "gemm 3");
    hip_check(out_fwd(c->a3, c->pb + kW4, c->p + kB4, rows, c->y, st), "output layer");
}

// gradient of the loss of the first n rows into c->g (loss added to c->loss)
void backward(prop_ctx* c, int n, int rows) {
    using namespace prop;
    hipStream_t st = c->stream;
    hip_check(out_bwd(c->y, c->yb, n, rows, c->a3, c->pb + kW4, c->z3, c->d3, c->g + kW4, c->g + kB4, c->loss, st),
              "output backward");
    Epi_args dw;
    dw.mode = kEpiDw;
    Epi_args dx;
    dx.mode = kEpiDx;
    // layer 3
    dw.out = c->g + kW3;
    hip_check(gemm(true, false, c->a2, kHidden, c->d3, kHidden, kHidden, kHidden, rows, dw, st), "dW3");
    hip_check(bias_grad(c->d3, rows, kHidden, c->g + kB3, st), "db3");
    dx.zmask = c->z2; dx.act = c->d2;
    hip_check(gemm(false, true, c->d3, kHidden, c->pb + kW3, kHidden, rows, kHidden, kHidden, dx, st), "dA2");
    // layer 2
    dw.out = c->g + kW2;
    hip_check(gemm(true, false, c->a1, kHidden, c->d2, kHidden, kHidden, kHidden, rows, dw, st), "dW2");
    hip_check(bias_grad(c->d2, rows, kHidden, c->g + kB2, st), "db2");
    dx.zmask = c->z1; dx.act = c->d1;
    hip_check(gemm(false, true, c->d2, kHidden, c->pb + kW2, kHidden, rows, kHidden, kHidden, dx, st), "dA1");
    // layer 1
    dw.out = c->g + kW1;
    hip_check(gemm(true, false, c->xb, kIn, c->d1, kHidden, kIn, kHidden, rows, dw, st), "dW1");
    hip_check(bias_grad(c->d1, rows, kHidden, c->g + kB1, st), "db1");
}

void check_x(const float* X, int64_t n) {
    if (n < 0) fail(CORR_EINVAL, "n < 0");
    if (n > 0 && !X) fail(CORR_EINVAL, "X_dev is NULL");
}

void upload_sync(void* dst, const void* src, size_t bytes, hipStream_t st) {
    hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

void set_params(prop_ctx* c, const float* host) {
    upload_sync(c->p, host, sizeof(float) * kNP, c->stream);
    hip_check(prop::round_params(c->p, kNP, c->pb, c->stream), "round");
    hip_check(hipMemsetAsync(c->m, 0, sizeof(float) * kNP, c->stream), "memset");
    hip_check(hipMemsetAsync(c->v, 0, sizeof(float) * kNP, c->stream), "memset");
    c->step = 0;
}

}  // namespace

extern "C" {

int prop_create(int32_t batch, uint64_t seed, void* hip_stream, prop_ctx** out) {
    prop_ctx* c = nullptr;
    int rc = guarded(nullptr, [&] {
        if (!out) fail(CORR_EINVAL, "out is NULL");
        *out = nullptr;
        if (batch < 64 || batch > 8192 || batch % 64) fail(CORR_EINVAL, "batch = %d; need a multiple of 64 in 64..8192", batch);
        c = new prop_ctx();
        c->stream = static_cast<hipStream_t>(hip_stream);
        c->batch = batch;
        c->seed = seed;
        auto& o = c->owned;
        c->p = dalloc<float>(o, kNP);
        c->g = dalloc<float>(o, kNP);
        c->m = dalloc<float>(o, kNP);
        c->v = dalloc<float>(o, kNP);
        c->pb = dalloc<uint16_t>(o, kNP);
        c->xb = dalloc<uint16_t>(o, (size_t)batch * prop::kIn);
        c->yb = dalloc<float>(o, batch);
        c->y = dalloc<float>(o, batch);
        c->z1 = dalloc<float>(o, (size_t)batch * prop::kHidden);
        c->z2 = dalloc<float>(o, (size_t)batch * prop::kHidden);
        c->z3 = dalloc<float>(o, (size_t)batch * prop::kHidden);
        c->a1 = dalloc<uint16_t>(o, (size_t)batch * prop::kHidden);
        c->a2 = dalloc<uint16_t>(o, (size_t)batch * prop::kHidden);
        c->a3 = dalloc<uint16_t>(o, (size_t)batch * prop::kHidden);
        c->d1 = dalloc<uint16_t>(o, (size_t)batch * prop::kHidden);
        c->d2 = dalloc<uint16_t>(o, (size_t)batch * prop::kHidden);
        c->d3 = dalloc<uint16_t>(o, (size_t)batch * prop::kHidden);
        c->loss = dalloc<float>(o, 1);
        // He-uniform weights, zero biases
        std::vector<float> init(kNP, 0.0f);
        std::mt19937_64 rng(seed);
        const int64_t wofs[4] = {kW1, kW2, kW3, kW4};
        const int fan_in[4] = {160, 256, 256, 256}, fan_out[4] = {256, 256, 256, 1};
        for (int l = 0; l < 4; ++l) {
            std::uniform_real_distribution<double> u(-std::sqrt(6.0 / fan_in[l]), std::sqrt(6.0 / fan_in[l]));
            for (int64_t i = 0; i < (int64_t)fan_in[l] * fan_out[l]; ++i) init[wofs[l] + i] = (float)u(rng);
        }
        set_params(c, init.data());
        *out = c;
    });
    if (rc != CORR_OK && c) prop_destroy(c);
    return rc;
}

int prop_descriptor(prop_ctx* c, const corr_ball* balls, int64_t n, float* desc_dev) {
    if (!c) { g_error = "prop_descriptor: NULL context"; return CORR_EINVAL; }
    return guarded(c, [&] {
        if (n < 1 || !balls || !desc_dev) fail(CORR_EINVAL, "need n >= 1 balls and an output");
        for (int64_t i = 0; i < n; ++i) {
            const corr_ball& b = balls[i];
            if (!std::isfinite(b.x) || !std::isfinite(b.y) || !std::isfinite(b.z) || !std::isfinite(b.w) ||
                !std::isfinite(b.r) || !(b.r > 0))
                fail(CORR_EINVAL, "ball %lld: non-finite value or radius <= 0", (long long)i);
            // the histogram is of volumes w r^3, normalised by their total: a
            // weight <= 0 has no volume (and a zero total no normalisation)
            if (!(b.w > 0)) fail(CORR_EINVAL, "ball %lld: weight must be > 0 for a volume descriptor", (long long)i);
        }
        std::vector<void*> tmp;
        try {
            double* d = dalloc<double>(tmp, (size_t)5 * n);
            upload_sync(d, balls, sizeof(double) * 5 * n, c->stream);
            hip_check(prop::descriptor(d, n, desc_dev, c->stream), "descriptor");
            hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
        } catch (...) {
            for (void* p : tmp) (void)hipFree(p);
            throw;
        }
        for (void* p : tmp) (void)hipFree(p);
    });
}

int prop_features(prop_ctx* c, const double* q, int64_t n, const float* da, const float* db, float* X) {
    if (!c) { g_error = "prop_features: NULL context"; return CORR_EINVAL; }
    return guarded(c, [&] {
        if (n < 0 || (n > 0 && (!q || !da || !db || !X))) fail(CORR_EINVAL, "bad arguments");
        for (int64_t i = 0; i < n; ++i) {
            double s = 0;
            for (int k = 0; k < 4; ++k) {
                if (!std::isfinite(q[4 * i + k])) fail(CORR_EINVAL, "quaternion %lld non-finite", (long long)i);
                s += q[4 * i + k] * q[4 * i + k];
            }
            if (std::sqrt(s) < 1e-12) fail(CORR_EINVAL, "quaternion %lld has norm < 1e-12", (long long)i);
        }
        if (n == 0) return;
        std::vector<void*> tmp;
        try {
            double* d = dalloc<double>(tmp, (size_t)4 * n);
            upload_sync(d, q, sizeof(double) * 4 * n, c->stream);
            hip_check(prop::features(d, n, da, db, X, c->stream), "features");
            hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
        } catch (...) {
            for (void* p : tmp) (void)hipFree(p);
            throw;
        }
        for (void* p : tmp) (void)hipFree(p);
    });
}

int prop_train(prop_ctx* c, const float* X, const float* y, int64_t n, int32_t epochs, float lr, float* loss_host) {
    if (!c) { g_error = "prop_train: NULL context"; return CORR_EINVAL; }
    return guarded(c, [&] {
        check_x(X, n);
        if (!y) fail(CORR_EINVAL, "y_dev is NULL");
        if (n < c->batch) fail(CORR_EINVAL, "n = %lld < batch = %d", (long long)n, c->batch);
        if (n > (int64_t)1 << 30) fail(CORR_EUNSUPPORTED, "n > 2^30");
        if (epochs < 0) fail(CORR_EINVAL, "epochs < 0");
        if (!(lr > 0) || !std::isfinite(lr)) fail(CORR_EINVAL, "lr must be finite and > 0");
        std::vector<void*> tmp;
        int* perm_host = nullptr;
        try {
            int* perm = dalloc<int>(tmp, (size_t)n);
            hip_check(hipHostMalloc((void**)&perm_host, sizeof(int) * n, hipHostMallocDefault), "hipHostMalloc");
            const int64_t nb = n / c->batch;
            for (int ep = 0; ep < epochs; ++ep) {
                hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");  // perm_host reuse
                std::iota(perm_host, perm_host + n, 0);
                std::mt19937_64 rng(c->seed * 1000003ull + (uint64_t)c->step + (uint64_t)ep);
                std::shuffle(perm_host, perm_host + n, rng);
                hip_check(hipMemcpyAsync(perm, perm_host, sizeof(int) * n, hipMemcpyHostToDevice, c->stream), "perm");
                hip_check(hipMemsetAsync(c->loss, 0, sizeof(float), c->stream), "memset");
                for (int64_t bi = 0; bi < nb; ++bi) {
                    hip_check(prop::gather(X, y, perm, bi * c->batch, c->batch, c->batch, c->xb, c->yb, c->stream),
                              "gather");
                    forward(c, c->batch);
                    backward(c, c->batch, c->batch);
                    c->step += 1;
                    const float c1 = 1.0f - (float)std::pow(0.9, (double)c->step);
                    const float c2 = 1.0f - (float)std::pow(0.999, (double)c->step);
                    hip_check(prop::adam(c->p, c->g, c->m, c->v, kNP, lr, 0.9f, 0.999f, 1e-8f, c1, c2, c->pb, c->stream),
                              "adam");
                }
                if (loss_host) {
                    float l = 0;
                    hip_check(hipMemcpyAsync(&l, c->loss, sizeof(float), hipMemcpyDeviceToHost, c->stream), "loss");
                    hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
                    loss_host[ep] = l / (float)std::max<int64_t>(nb, 1);
                }
            }
            hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
        } catch (...) {
            (void)hipStreamSynchronize(c->stream);
            for (void* p : tmp) (void)hipFree(p);
            if (perm_host) (void)hipHostFree(perm_host);
            throw;
        }
        for (void* p : tmp) (void)hipFree(p);
        if (perm_host) (void)hipHostFree(perm_host);
    });
}

int prop_predict(prop_ctx* c, const float* X, int64_t n, float* y_out) {
    if (!c) { g_error = "prop_predict: NULL context"; return CORR_EINVAL; }
    return guarded(c, [&] {
        check_x(X, n);
        if (n > 0 && !y_out) fail(CORR_EINVAL, "y_dev is NULL");
        for (int64_t r0 = 0; r0 < n; r0 += c->batch) {
            const int rows = (int)std::min<int64_t>(c->batch, n - r0);
            hip_check(prop::gather(X, nullptr, nullptr, r0, rows, c->batch, c->xb, c->yb, c->stream), "gather");
            forward(c, c->batch);
            hip_check(hipMemcpyAsync(y_out + r0, c->y, sizeof(float) * rows, hipMemcpyDeviceToDevice, c->stream), "copy");
        }
    });
}

int prop_rank(prop_ctx* c, const float* X, int64_t n, int32_t k, int64_t* idx) {
    if (!c) { g_error = "prop_rank: NULL context"; return CORR_EINVAL; }
    return guarded(c, [&] {
        check_x(X, n);
        if (n < 1 || n > prop::kRankMax) fail(CORR_EUNSUPPORTED, "n = %lld; rank supports 1..%d", (long long)n, prop::kRankMax);
        if (k < 1 || k > n) fail(CORR_EINVAL, "k = %d outside 1..n", k);
        if (!idx) fail(CORR_EINVAL, "idx_dev is NULL");
        std::vector<void*> tmp;
        try {
            float* yy = dalloc<float>(tmp, (size_t)n);
            for (int64_t r0 = 0; r0 < n; r0 += c->batch) {
                const int rows = (int)std::min<int64_t>(c->batch, n - r0);
                hip_check(prop::gather(X, nullptr, nullptr, r0, rows, c->batch, c->xb, c->yb, c->stream), "gather");
                forward(c, c->batch);
                hip_check(hipMemcpyAsync(yy + r0, c->y, sizeof(float) * rows, hipMemcpyDeviceToDevice, c->stream), "copy");
            }
            hip_check(prop::topk(yy, (int)n, k, idx, c->stream), "topk");
            hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
        } catch (...) {
            (void)hipStreamSynchronize(c->stream);
            for (void* p : tmp) (void)hipFree(p);
            throw;
        }
        for (void* p : tmp) (void)hipFree(p);
    });
}

int prop_gradient(prop_ctx* c, const float* X, const float* y, int64_t n, float* grads_host) {
    if (!c) { g_error = "prop_gradient: NULL context"; return CORR_EINVAL; }
    return guarded(c, [&] {
        check_x(X, n);
        if (n < 1 || n > c->batch) fail(CORR_EINVAL, "n must be in 1..batch");
        if (!y || !grads_host) fail(CORR_EINVAL, "NULL argument");
        hip_check(prop::gather(X, y, nullptr, 0, (int)n, c->batch, c->xb, c->yb, c->stream), "gather");
        forward(c, c->batch);
        hip_check(hipMemsetAsync(c->loss, 0, sizeof(float), c->stream), "memset");
        backward(c, (int)n, c->batch);
        hip_check(hipMemcpyAsync(grads_host, c->g, sizeof(float) * kNP, hipMemcpyDeviceToHost, c->stream), "copy");
        hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    });
}

int prop_get_params(prop_ctx* c, float* host_out) {
    if (!c) { g_error = "prop_get_params: NULL context"; return CORR_EINVAL; }
    return guarded(c, [&] {
        if (!host_out) fail(CORR_EINVAL, "NULL output");
        hip_check(hipMemcpyAsync(host_out, c->p, sizeof(float) * kNP, hipMemcpyDeviceToHost, c->stream), "copy");
        hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    });
}

int prop_set_params(prop_ctx* c, const float* host_in) {
    if (!c) { g_error = "prop_set_params: NULL context"; return CORR_EINVAL; }
    return guarded(c, [&] {
        if (!host_in) fail(CORR_EINVAL, "NULL input");
        for (int64_t i = 0; i < kNP; ++i)
            if (!std::isfinite(host_in[i])) fail(CORR_EINVAL, "parameter %lld is not finite", (long long)i);
        set_params(c, host_in);
    });
}

int prop_destroy(prop_ctx* c) {
    if (!c) return CORR_OK;
    (void)hipStreamSynchronize(c->stream);
    for (void* p : c->owned) (void)hipFree(p);
    delete c;
    return CORR_OK;
}

const char* prop_last_error(const prop_ctx* c) { return c ? c->err.c_str() : g_error.c_str(); }

}  // extern "C"

// Internal interface between prop_host.cpp and prop_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace prop {

constexpr int kIn = 160;
constexpr int kHidden = 256;
constexpr int kBins = 64;
constexpr int kRot = 9;  // rotation-matrix entries; the inputs hold R, sin(pi R), cos(pi R)
constexpr int kRankMax = 8192;

constexpr int kEpiHidden = 0;  // z = acc + bias -> z (f32), relu(z) -> bf16
constexpr int kEpiDx = 1;      // acc masked by (zmask > 0) -> bf16
constexpr int kEpiDw = 2;      // acc -> f32

struct Epi_args {
    int mode = kEpiDw;
    const float* bias = nullptr;
    float* z = nullptr;
    uint16_t* act = nullptr;
    const float* zmask = nullptr;
    float* out = nullptr;
};

// C[M][N] = op(A) op(B) with bf16 operands on the matrix cores, FP32 sums.
hipError_t gemm(bool ta, bool tb, const uint16_t* A, int lda, const uint16_t* B, int ldb, int M, int N, int K,
                const Epi_args& e, hipStream_t st);
hipError_t out_fwd(const uint16_t* a, const uint16_t* w, const float* b4, int rows, float* y, hipStream_t st);
hipError_t out_bwd(const float* y, const float* t, int n, int rows, const uint16_t* a3, const uint16_t* w4,
                   const float* z3, uint16_t* dz3, float* g_w4, float* g_b4, float* loss, hipStream_t st);
hipError_t bias_grad(const uint16_t* dz, int rows, int cols, float* db, hipStream_t st);
hipError_t gather(const float* X, const float* y, const int* perm, int64_t start, int n, int rows, uint16_t* xb,
                  float* yb, hipStream_t st);
hipError_t adam(float* p, const float* g, float* m, float* v, int64_t np, float lr, float b1, float b2, float eps,
                float c1, float c2, uint16_t* pb, hipStream_t st);
hipError_t round_params(const float* p, int64_t np, uint16_t* pb, hipStream_t st);
hipError_t features(const double* q, int64_t n, const float* da, const float* db, float* X, hipStream_t st);
hipError_t descriptor(const double* balls, int64_t n, float* out, hipStream_t st);
hipError_t topk(const float* y, int n, int k, int64_t* idx, hipStream_t st);

}  // namespace prop

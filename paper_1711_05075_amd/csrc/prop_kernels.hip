// gfx950 kernels of the rotation-proposal network: bfloat16 matrix-core GEMMs
// with FP32 accumulation (v_mfma_f32_32x32x8_bf16), their epilogues, the output
// layer, the loss, Adam, descriptors and top-k selection.
#include "prop_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>

namespace prop {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kT = 256;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float -> bfloat16, round to nearest, ties to even (NaN kept a quiet NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// C = op(A) op(B) on the matrix cores.  A(i, k) = TA ? A[k*lda + i] : A[i*lda + k],
// B(k, j) = TB ? B[j*ldb + k] : B[k*ldb + j]; K a multiple of 32; rows and
// columns past M and N are masked.
// A workgroup of four waves computes a 64 x 64 tile, each wave a 32 x 32 block
// with one 32x32x8 bf16 MFMA per 8-deep slice of K.  Operand lanes (per the
// instruction's layout): A lane l holds rows l % 32, k = 4 (l / 32) .. +3;
// B lane l holds column l % 32, the same k; accumulator register r of lane l
// is row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
// ---------------------------------------------------------------------------
struct Epi {
    int mode;              // kEpiHidden, kEpiDx, kEpiDw
    const float* bias;     // [N]            (hidden)
    float* z;              // [M][N] f32     (hidden: pre-activation out)
    uint16_t* act;         // [M][N] bf16    (hidden: ReLU out; dx: masked gradient out)
    const float* zmask;    // [M][N] f32     (dx: pre-activation of the layer below)
    float* out;            // [M][N] f32     (dw)
};

template <bool TA, bool TB>
__global__ __launch_bounds__(kT) void k_gemm(const uint16_t* __restrict__ A, int lda, const uint16_t* __restrict__ B,
                                             int ldb, int M, int N, int K, Epi e) {
    __shared__ uint16_t sA[64][40];  // [i][k], padded
    __shared__ uint16_t sB[64][40];  // [j][k], padded
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    for (int k0 = 0; k0 < K; k0 += 32) {
        // 64 x 32 elements of each operand, 8 per thread
        for (int t = tid; t < 64 * 32; t += kT) {
            int i, k;
            if (TA) { k = t >> 6; i = t & 63; } else { i = t >> 5; k = t & 31; }
            const bool ia = i0 + i < M;  // rows past M read as zero
            sA[i][k] = !ia ? (uint16_t)0
                           : TA ? A[(size_t)(k0 + k) * lda + i0 + i] : A[(size_t)(i0 + i) * lda + k0 + k];
            int j, kb;
            if (TB) { j = t >> 5; kb = t & 31; } else { kb = t >> 6; j = t & 63; }
            const bool jb = j0 + j < N;
            sB[j][kb] = !jb ? (uint16_t)0
                            : TB ? B[(size_t)(j0 + j) * ldb + k0 + kb] : B[(size_t)(k0 + kb) * ldb + j0 + j];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 32; kk += 8) {
            const int ka = kk + 4 * (lane >> 5);
            bf16x4 a, b;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = (short)sA[32 * wr + (lane & 31)][ka + u];
                b[u] = (short)sB[32 * wc + (lane & 31)][ka + u];
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    const int j = j0 + 32 * wc + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = i0 + 32 * wr + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i >= M || j >= N) continue;
        const size_t o = (size_t)i * N + j;
        const float v = acc[r];
        if (e.mode == kEpiHidden) {
            const float z = v + e.bias[j];
            e.z[o] = z;
            e.act[o] = f2bf(z > 0.f ? z : 0.f);
        } else if (e.mode == kEpiDx) {
            e.act[o] = f2bf(e.zmask[o] > 0.f ? v : 0.f);
        } else {
            e.out[o] = v;
        }
    }
}

// Output layer y[b] = sum_k a[b][k] w[k] + b4 (bf16 inputs, FP32 sum): one wave per row.
__global__ __launch_bounds__(kT) void k_out_fwd(const uint16_t* __restrict__ a, const uint16_t* __restrict__ w,
                                                const float* __restrict__ b4, int rows, float* __restrict__ y) {
    const int row = blockIdx.x * (kT / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= rows) return;
    float s = 0.f;
    for (int k = lane; k < kHidden; k += 64) s += bf2f(a[(size_t)row * kHidden + k]) * bf2f(w[k]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) y[row] = s + b4[0];
}

// Loss and output-layer backward for one batch of `rows` (n real, rest padding):
// dz4 = 2 (y - t) / n; dA3 = dz4 w4 masked by z3 > 0 -> bf16; dW4 = sum_b a3 dz4;
// db4 = sum_b dz4; loss += sum_b (y - t)^2 / n.  One workgroup.
__global__ __launch_bounds__(kT) void k_out_bwd(const float* __restrict__ y, const float* __restrict__ t, int n,
                                                int rows, const uint16_t* __restrict__ a3,
                                                const uint16_t* __restrict__ w4, const float* __restrict__ z3,
                                                uint16_t* __restrict__ dz3, float* __restrict__ g_w4,
                                                float* __restrict__ g_b4, float* __restrict__ loss) {
    __shared__ float dz[8192];
    __shared__ float red[kT];
    float l2 = 0.f, sdz = 0.f;
    for (int b = threadIdx.x; b < rows; b += kT) {
        const float d = b < n ? y[b] - t[b] : 0.f;
        dz[b] = 2.f * d / (float)n;
        l2 += d * d;
        sdz += dz[b];
    }
    __syncthreads();
    // dW4[k] for k = threadIdx.x (kHidden == kT)
    {
        const int k = threadIdx.x;
        float s = 0.f;
        for (int b = 0; b < rows; ++b) s += bf2f(a3[(size_t)b * kHidden + k]) * dz[b];
        g_w4[k] = s;
    }
    for (int idx = threadIdx.x; idx < rows * kHidden; idx += kT) {
        const int b = idx / kHidden, k = idx % kHidden;
        const float v = dz[b] * bf2f(w4[k]);
        dz3[idx] = f2bf(z3[idx] > 0.f ? v : 0.f);
    }
    red[threadIdx.x] = l2;
    __syncthreads();
    for (int off = kT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] += red[0] / (float)n;
    __syncthreads();
    red[threadIdx.x] = sdz;
    __syncthreads();
    for (int off = kT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) g_b4[0] = red[0];
}

// Bias gradient db[j] = sum_b dz[b][j] (bf16 gradients, FP32 sum).
__global__ __launch_bounds__(kT) void k_bias_grad(const uint16_t* __restrict__ dz, int rows, int cols,
                                                  float* __restrict__ db) {
    const int j = blockIdx.x * kT + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int b = 0; b < rows; ++b) s += bf2f(dz[(size_t)b * cols + j]);
    db[j] = s;
}

// Gather a mini-batch: rows perm[start + b] of X (rounded to bf16) and of y;
// rows past n are zero (and excluded from the loss by n).
__global__ __launch_bounds__(kT) void k_gather(const float* __restrict__ X, const float* __restrict__ y,
                                               const int* __restrict__ perm, int64_t start, int n, int rows,
                                               uint16_t* __restrict__ xb, float* __restrict__ yb) {
    const int idx = blockIdx.x * kT + threadIdx.x;
    if (idx >= rows * kIn) return;
    const int b = idx / kIn, k = idx % kIn;
    if (b < n) {
        const int64_t src = perm ? perm[start + b] : start + b;
        xb[idx] = f2bf(X[src * kIn + k]);
        if (k == 0) yb[b] = y ? y[src] : 0.f;
    } else {
        xb[idx] = 0;
        if (k == 0) yb[b] = 0.f;
    }
}

// Adam on the FP32 master parameters; weights re-rounded to their bf16 copies.
__global__ __launch_bounds__(kT) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                             float* __restrict__ v, int64_t np, float lr, float b1, float b2,
                                             float eps, float c1, float c2, uint16_t* __restrict__ pb) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    pb[i] = f2bf(pi);
}

__global__ __launch_bounds__(kT) void k_round(const float* __restrict__ p, int64_t np, uint16_t* __restrict__ pb) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < np) pb[i] = f2bf(p[i]);
}

// Network inputs: canonical quaternion (w >= 0, unit), both descriptors, zeros.
__global__ __launch_bounds__(kT) void k_features(const double* __restrict__ q, int64_t n,
                                                 const float* __restrict__ da, const float* __restrict__ db,
                                                 float* __restrict__ X) {
    const int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (idx >= n * kIn) return;
    const int64_t r = idx / kIn;
    const int k = (int)(idx % kIn);
    float v = 0.f;
    if (k < 3 * kRot) {
        // entry e of R(q), built in FP64 from the normalised quaternion (the same
        // matrix for q and -q), then R_e, sin(pi R_e) or cos(pi R_e)
        const double* qq = q + 4 * r;
        const double nn = qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2] + qq[3] * qq[3];
        const double w = qq[0], x = qq[1], y = qq[2], z = qq[3], s = 2.0 / nn;
        const int e = k % kRot;
        double m;
        switch (e) {
            case 0: m = 1.0 - s * (y * y + z * z); break;
            case 1: m = s * (x * y - w * z); break;
            case 2: m = s * (x * z + w * y); break;
            case 3: m = s * (x * y + w * z); break;
            case 4: m = 1.0 - s * (x * x + z * z); break;
            case 5: m = s * (y * z - w * x); break;
            case 6: m = s * (x * z - w * y); break;
            case 7: m = s * (y * z + w * x); break;
            default: m = 1.0 - s * (x * x + y * y); break;
        }
        const int part = k / kRot;
        v = (float)(part == 0 ? m : part == 1 ? sin(M_PI * m) : cos(M_PI * m));
    } else if (k < 3 * kRot + kBins) {
        v = (float)kBins * da[k - 3 * kRot];
    } else if (k < 3 * kRot + 2 * kBins) {
        v = (float)kBins * db[k - 3 * kRot - kBins];
    }
    X[idx] = v;
}

// Descriptor of one ball set: volume-weighted centroid (FP64), then the
// volume histogram over centre distance with exact fixed-point sums.
__global__ __launch_bounds__(1024) void k_descriptor(const double* __restrict__ balls, int64_t n,
                                                     float* __restrict__ out) {
    __shared__ double red[4][1024];
    __shared__ unsigned long long hist[kBins];
    __shared__ double total;
    double sx = 0, sy = 0, sz = 0, sv = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        const double* b = balls + 5 * i;
        const double v = b[4] * b[3] * b[3] * b[3];
        sx += v * b[0];
        sy += v * b[1];
        sz += v * b[2];
        sv += v;
    }
    red[0][threadIdx.x] = sx;
    red[1][threadIdx.x] = sy;
    red[2][threadIdx.x] = sz;
    red[3][threadIdx.x] = sv;
    if (threadIdx.x < kBins) hist[threadIdx.x] = 0ull;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + off];
        __syncthreads();
    }
    const double cx = red[0][0] / red[3][0], cy = red[1][0] / red[3][0], cz = red[2][0] / red[3][0];
    if (threadIdx.x == 0) total = red[3][0];
    __syncthreads();
    // fixed point: every volume as a fraction of the total, 2^62 scale
    const double scale = 4611686018427387904.0 / total;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        const double* b = balls + 5 * i;
        const double v = b[4] * b[3] * b[3] * b[3];
        const double dx = b[0] - cx, dy = b[1] - cy, dz = b[2] - cz;
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        int bin = (int)(d * kBins);
        if (bin > kBins - 1) bin = kBins - 1;
        atomicAdd(&hist[bin], (unsigned long long)llrint(v * scale));
    }
    __syncthreads();
    if (threadIdx.x < kBins) {
        unsigned long long s = 0;
        for (int k = 0; k < kBins; ++k) s += hist[k];
        out[threadIdx.x] = (float)((double)hist[threadIdx.x] / (double)s);
    }
}

// Top-k by descending score (NaN lowest; ties: lower index first) with one
// workgroup: a bitonic sort of (score, index) keys in LDS, n <= kRankMax.
__device__ __forceinline__ bool key_before(float a, int ia, float b, int ib) {
    if (a != a) a = -INFINITY;
    if (b != b) b = -INFINITY;
    return a > b || (a == b && ia < ib);
}

__global__ __launch_bounds__(1024) void k_topk(const float* __restrict__ y, int n, int k, int64_t* __restrict__ idx) {
    __shared__ float key[kRankMax];
    __shared__ int id[kRankMax];
    int p2 = 1;
    while (p2 < n) p2 <<= 1;
    for (int t = threadIdx.x; t < p2; t += 1024) {
        key[t] = t < n ? y[t] : -INFINITY;
        id[t] = t < n ? t : 0x7fffffff;
    }
    __syncthreads();
    for (int size = 2; size <= p2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < p2; t += 1024) {
                const int u = t ^ stride;
                if (u > t) {
                    const bool up = (t & size) == 0;  // this run sorts "best first"
                    const bool swap = up ? key_before(key[u], id[u], key[t], id[t])
                                         : key_before(key[t], id[t], key[u], id[u]);
                    if (swap) {
                        const float kk = key[t];
                        key[t] = key[u];
                        key[u] = kk;
                        const int ii = id[t];
                        id[t] = id[u];
                        id[u] = ii;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < k; t += 1024) idx[t] = id[t];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t gemm(bool ta, bool tb, const uint16_t* A, int lda, const uint16_t* B, int ldb, int M, int N, int K,
                const Epi_args& a, hipStream_t st) {
    Epi e{a.mode, a.bias, a.z, a.act, a.zmask, a.out};
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    if (!ta && !tb) hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(kT), 0, st, A, lda, B, ldb, M, N, K, e);
    else if (!ta && tb) hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(kT), 0, st, A, lda, B, ldb, M, N, K, e);
    else if (ta && !tb) hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(kT), 0, st, A, lda, B, ldb, M, N, K, e);
    else hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(kT), 0, st, A, lda, B, ldb, M, N, K, e);
    return hipGetLastError();
}

hipError_t out_fwd(const uint16_t* a, const uint16_t* w, const float* b4, int rows, float* y, hipStream_t st) {
    hipLaunchKernelGGL(k_out_fwd, dim3((rows + 3) / 4), dim3(kT), 0, st, a, w, b4, rows, y);
    return hipGetLastError();
}

hipError_t out_bwd(const float* y, const float* t, int n, int rows, const uint16_t* a3, const uint16_t* w4,
                   const float* z3, uint16_t* dz3, float* g_w4, float* g_b4, float* loss, hipStream_t st) {
    hipLaunchKernelGGL(k_out_bwd, dim3(1), dim3(kT), 0, st, y, t, n, rows, a3, w4, z3, dz3, g_w4, g_b4, loss);
    return hipGetLastError();
}

hipError_t bias_grad(const uint16_t* dz, int rows, int cols, float* db, hipStream_t st) {
    hipLaunchKernelGGL(k_bias_grad, dim3((cols + kT - 1) / kT), dim3(kT), 0, st, dz, rows, cols, db);
    return hipGetLastError();
}

hipError_t gather(const float* X, const float* y, const int* perm, int64_t start, int n, int rows, uint16_t* xb,
                  float* yb, hipStream_t st) {
    hipLaunchKernelGGL(k_gather, dim3((rows * kIn + kT - 1) / kT), dim3(kT), 0, st, X, y, perm, start, n, rows, xb,
                       yb);
    return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m, float* v, int64_t np, float lr, float b1, float b2, float eps,
                float c1, float c2, uint16_t* pb, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((np + kT - 1) / kT)), dim3(kT), 0, st, p, g, m, v, np, lr, b1, b2, eps,
                       c1, c2, pb);
    return hipGetLastError();
}

hipError_t round_params(const float* p, int64_t np, uint16_t* pb, hipStream_t st) {
    hipLaunchKernelGGL(k_round, dim3((unsigned)((np + kT - 1) / kT)), dim3(kT), 0, st, p, np, pb);
    return hipGetLastError();
}

hipError_t features(const double* q, int64_t n, const float* da, const float* db, float* X, hipStream_t st) {
    hipLaunchKernelGGL(k_features, dim3((unsigned)((n * kIn + kT - 1) / kT)), dim3(kT), 0, st, q, n, da, db, X);
    return hipGetLastError();
}

hipError_t descriptor(const double* balls, int64_t n, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_descriptor, dim3(1), dim3(1024), 0, st, balls, n, out);
    return hipGetLastError();
}

hipError_t topk(const float* y, int n, int k, int64_t* idx, hipStream_t st) {
    hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, st, y, n, k, idx);
    return hipGetLastError();
}

}  // namespace prop

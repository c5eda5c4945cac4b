// gfx950 kernels of the ball-union correlation pipeline.
//
// Shape spectrum (Behandish & Ilies, Sec. 2.5 eq. eq_rhoPhat weighted by the
// ball transform) by a type-1 nonequispaced FFT:
//   a0  turn the knots (App. B action, rotation built in FP64) and place them on
//       an oversampled periodic grid of m = sigma*n cells per axis;
//   a1  spread each knot's q radius-expansion weights with a separable
//       Kaiser-Bessel window of w cells;
//   a2  forward FFT of each component, pruned to the kept modes |m_d| < n/2;
//   a3  sum the components against the ball-transform table and divide by the
//       window's transform (both tables built in FP64).
// Correlation (Sec. 3.2 eq. eq_ccghat):
//   a4  S = F_A conj(F_RB) exp(i k.origin) / L^3 on the half cube of modes;
//   a5  inverse FFT to the n^3 translation grid, with per-rotation peaks.
//
// Column FFTs run in LDS as Stockham autosort passes of radix 8, 4 and 2 (each
// thread does one radix-R butterfly per pass in registers), over a batch of
// columns so that every HBM access is a contiguous row segment.
#include "corr_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>

namespace corr {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// a * (SIGN * i)
template <int SIGN>
__device__ __forceinline__ float2 mul_si(float2 a) {
    return SIGN < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

template <int SIGN>
__device__ __forceinline__ void dft2(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

// X_s = sum_r v_r exp(SIGN 2 pi i r s / 4)
template <int SIGN>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
    float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
    float2 t2 = cadd(a1, a3), t3 = mul_si<SIGN>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <int SIGN>
__device__ __forceinline__ void dft8(float2* v) {
    // even / odd halves, then combine with exp(SIGN 2 pi i k / 8)
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<SIGN>(e0, e1, e2, e3);
    dft4<SIGN>(o0, o1, o2, o3);
    const float h = 0.70710678118654752440f;
    float2 w1o = cmul(o1, make_float2(h, SIGN * h));
    float2 w2o = mul_si<SIGN>(o2);
    float2 w3o = cmul(o3, make_float2(-h, SIGN * h));
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, w1o);
    v[5] = csub(e1, w1o);
    v[2] = cadd(e2, w2o);
    v[6] = csub(e2, w2o);
    v[3] = cadd(e3, w3o);
    v[7] = csub(e3, w3o);
}

// One Stockham pass of radix R over `cols` columns of length `len`; element
// (i, c) of a column batch lives at buf[i * si + c * sc].  tw[j] = exp(-2 pi i j / len).
template <int R, int SIGN>
__device__ __forceinline__ void stockham_pass(const float2* __restrict__ src, float2* __restrict__ dst,
                                              int si, int sc, int len, int cols, int ns,
                                              const float2* __restrict__ tw) {
    const int nb = len / R;
    const int tws = len / (ns * R);
    for (int t = threadIdx.x; t < nb * cols; t += blockDim.x) {
        const int c = t % cols, j = t / cols;
        const int k = j % ns;
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[(j + r * nb) * si + c * sc];
        if (k) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tw[r * k * tws];
                if (SIGN > 0) w.y = -w.y;
                v[r] = cmul(v[r], w);
            }
        }
        if (R == 8) dft8<SIGN>(v);
        else if (R == 4) dft4<SIGN>(v[0], v[1], v[2], v[3]);
        else dft2<SIGN>(v);
        const int o = (j / ns) * ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[(o + r * ns) * si + c * sc] = v[r];
    }
}

// Unnormalised DFT of every column (sum_i x_i exp(SIGN 2 pi i i s / len)) with
// a and b as ping-pong buffers; returns the buffer that holds the result.
// Must be entered by the whole workgroup after the input is visible in `a`.
template <int SIGN>
__device__ float2* fft_cols(float2* a, float2* b, int si, int sc, int len, int cols,
                            const float2* __restrict__ tw) {
    int ns = 1;
    while (ns < len) {
        const int rem = len / ns;
        if (rem >= 8) {
            stockham_pass<8, SIGN>(a, b, si, sc, len, cols, ns, tw);
            ns *= 8;
        } else if (rem == 4) {
            stockham_pass<4, SIGN>(a, b, si, sc, len, cols, ns, tw);
            ns *= 4;
        } else {
            stockham_pass<2, SIGN>(a, b, si, sc, len, cols, ns, tw);
            ns *= 2;
        }
        __syncthreads();
        float2* t = a;
        a = b;
        b = t;
    }
    return a;
}

__device__ __forceinline__ int signed_mode(int i, int n) { return i < n / 2 ? i : i - n; }

// Normalised Kaiser-Bessel window at offset u (|u| <= w/2) in spreading cells.
__device__ __forceinline__ float kb_window(float u, float two_over_w, float beta, float inv_i0beta) {
    float x = u * two_over_w;
    float s = fmaxf(1.0f - x * x, 0.0f);
    return cyl_bessel_i0f(beta * sqrtf(s)) * inv_i0beta;
}

// ---------------------------------------------------------------------------
// FP64 tables
// ---------------------------------------------------------------------------

// Deconvolution 1/phihat(m/M) of the normalised window, per FFT index of an
// n-point axis, and the per-axis product factor D(m) exp(i k_m o_d) / L.
// phihat(nu) = w sinh(sqrt(beta^2 - (pi w nu)^2)) / sqrt(...) / I0(beta).
__global__ void k_deconv_tables(int n, int m, int w, double beta, double box, double o0, double o1,
                                double o2, double* __restrict__ deconv, double2* __restrict__ phase) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int md = signed_mode(i, n);
    if (md == -n / 2) {
        deconv[i] = 0.0;
        for (int d = 0; d < 3; ++d) phase[d * n + i] = make_double2(0.0, 0.0);
        return;
    }
    double nu = (double)md / (double)m;
    double x = M_PI * w * nu;
    double s = beta * beta - x * x;
    double ph;
    if (s > 0) {
        double r = sqrt(s);
        ph = w * sinh(r) / r;
    } else if (s < 0) {
        double r = sqrt(-s);
        ph = w * sin(r) / r;
    } else {
        ph = (double)w;
    }
    ph /= cyl_bessel_i0(beta);
    double dv = 1.0 / ph;
    deconv[i] = dv;
    double k = 2.0 * M_PI * md / box;
    const double org[3] = {o0, o1, o2};
    for (int d = 0; d < 3; ++d) {
        double sn, cs;
        sincos(k * org[d], &sn, &cs);
        phase[d * n + i] = make_double2(dv * cs / box, dv * sn / box);
    }
}

// (sin x - x cos x) / x^3 * 3, with its Taylor series below x = 0.5 where the
// closed form cancels.
__device__ double ball_shape(double x) {
    if (x < 0.5) {
        double x2 = x * x;
        return 3.0 * (1.0 / 3.0 - x2 * (1.0 / 30.0 - x2 * (1.0 / 840.0 - x2 * (1.0 / 45360.0 - x2 * (1.0 / 3991680.0 - x2 * (1.0 / 518918400.0))))));
    }
    double sn, cs;
    sincos(x, &sn, &cs);
    return 3.0 * (sn - x * cs) / (x * x * x);
}

// vtab[c][m2] = (4 pi / 3) rhi^3 sum_b (r_b / rhi)^3 Phi(k r_b) basis[b][c], k = dk sqrt(m2):
// the k-factor of the separable radius expansion of the ball transform.
__global__ void k_ball_table(int m2n, double dk, const double* __restrict__ nodes,
                             const double* __restrict__ basis, int p, int q, double rhi,
                             float* __restrict__ vtab) {
    int m2 = blockIdx.x * blockDim.x + threadIdx.x;
    if (m2 >= m2n) return;
    double k = dk * sqrt((double)m2);
    double acc[32];
    for (int c = 0; c < q; ++c) acc[c] = 0.0;
    for (int b = 0; b < p; ++b) {
        double rr = nodes[b] / rhi;
        double f = rr * rr * rr * ball_shape(k * nodes[b]);
        for (int c = 0; c < q; ++c) acc[c] += f * basis[b * q + c];
    }
    double scale = 4.0 * M_PI / 3.0 * rhi * rhi * rhi;
    for (int c = 0; c < q; ++c) vtab[(size_t)c * m2n + m2] = (float)(scale * acc[c]);
}

// ---------------------------------------------------------------------------
// a0: rotate + place
// ---------------------------------------------------------------------------

// Knot record: fractional offsets within the cell (x, y, z) and the cell index
// packed as cx | cy << 10 | cz << 20 (m <= 512).  The position is formed in
// FP64 so that the fraction keeps full float precision.
__global__ void k_rotate(const double* __restrict__ quats, const double* __restrict__ pos, int64_t nk,
                         double inv_hf, int m, float4* __restrict__ knots) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int s = blockIdx.y;
    if (j >= nk) return;
    const double* q = quats + 4 * s;
    double nn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double w = q[0] / nn, x = q[1] / nn, y = q[2] / nn, z = q[3] / nn;
    double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),     2 * (x * z + w * y),
                   2 * (x * y + w * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                   2 * (x * z - w * y),     2 * (y * z + w * x),     1 - 2 * (x * x + y * y)};
    double px = pos[3 * j], py = pos[3 * j + 1], pz = pos[3 * j + 2];
    double u[3] = {(R[0] * px + R[1] * py + R[2] * pz) * inv_hf, (R[3] * px + R[4] * py + R[5] * pz) * inv_hf,
                   (R[6] * px + R[7] * py + R[8] * pz) * inv_hf};
    float f[3];
    int c[3];
    for (int d = 0; d < 3; ++d) {
        double fl = floor(u[d]);
        f[d] = (float)(u[d] - fl);
        long long ci = (long long)fl % m;
        if (ci < 0) ci += m;
        c[d] = (int)ci;
        if (f[d] >= 1.0f) {  // rounding up to 1 moves to the next cell
            f[d] = 0.0f;
            c[d] = (c[d] + 1) % m;
        }
    }
    knots[(int64_t)s * nk + j] = make_float4(f[0], f[1], f[2], __int_as_float(c[0] | (c[1] << 10) | (c[2] << 20)));
}

__global__ void k_zero(float4* __restrict__ p, size_t n4) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n4; i += stride) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// ---------------------------------------------------------------------------
// a1: spreading (one workgroup of 64 lanes per knot; lanes own (dy, dz) rows)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_spread(const float4* __restrict__ knots, int64_t nk,
                                               const float* __restrict__ wts, int q, int m, int w,
                                               float beta, float inv_i0beta, float* __restrict__ fine) {
    int64_t j = blockIdx.x;
    int s = blockIdx.y;
    float4 kn = knots[(int64_t)s * nk + j];
    int packed = __float_as_int(kn.w);
    int cx = packed & 1023, cy = (packed >> 10) & 1023, cz = (packed >> 20) & 1023;
    const float tw = 2.0f / (float)w;
    const int lo = w / 2 - 1;
    float wx[16];
    for (int d = 0; d < w; ++d) wx[d] = kb_window(kn.x - (float)(d - lo), tw, beta, inv_i0beta);
    const size_t m3 = (size_t)m * m * m;
    for (int t = threadIdx.x; t < w * w; t += blockDim.x) {
        int dy = t % w, dz = t / w;
        float wyz = kb_window(kn.y - (float)(dy - lo), tw, beta, inv_i0beta) *
                    kb_window(kn.z - (float)(dz - lo), tw, beta, inv_i0beta);
        int yy = (cy + dy - lo + m) & (m - 1);
        int zz = (cz + dz - lo + m) & (m - 1);
        for (int c = 0; c < q; ++c) {
            float wq = wts[(size_t)c * nk + j] * wyz;
            float* row = fine + ((size_t)s * q + c) * m3 + ((size_t)zz * m + yy) * m;
            for (int dx = 0; dx < w; ++dx) {
                int xx = (cx + dx - lo + m) & (m - 1);
                atomicAdd(row + xx, wq * wx[dx]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// a2: x pass.  Two real lines are packed into one complex column, transformed
// together and separated: X1 = (Z_m + conj Z_{M-m}) / 2, X2 = (Z_m - conj Z_{M-m}) / 2i.
// LDS layout [column][i] with a padded column stride.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_fft_x(const float* __restrict__ fine, float2* __restrict__ out,
                                                    int m, int half, int cols, const float2* __restrict__ tw) {
    extern __shared__ float2 lds[];
    const int sc = m + 1;
    float2* a = lds;
    float2* b = lds + cols * sc;
    const size_t slab = blockIdx.y;
    const size_t line0 = (size_t)blockIdx.x * 2 * cols;
    const float* src = fine + slab * (size_t)m * m * m + line0 * m;
    const int nx4 = m / 4;
    for (int t = threadIdx.x; t < cols * nx4; t += blockDim.x) {
        int c = t / nx4, x4 = t % nx4;
        float4 r0 = *reinterpret_cast<const float4*>(src + (size_t)(2 * c) * m + 4 * x4);
        float4 r1 = *reinterpret_cast<const float4*>(src + (size_t)(2 * c + 1) * m + 4 * x4);
        float2* d = a + c * sc + 4 * x4;
        d[0] = make_float2(r0.x, r1.x);
        d[1] = make_float2(r0.y, r1.y);
        d[2] = make_float2(r0.z, r1.z);
        d[3] = make_float2(r0.w, r1.w);
    }
    __syncthreads();
    float2* res = fft_cols<-1>(a, b, 1, sc, m, cols, tw);
    float2* dst = out + slab * (size_t)m * m * half + line0 * half;
    for (int t = threadIdx.x; t < 2 * cols * half; t += blockDim.x) {
        int l = t / half, mm = t % half;
        int c = l >> 1;
        float2 z1 = res[c * sc + mm];
        float2 z2 = res[c * sc + ((m - mm) & (m - 1))];
        float2 o = (l & 1) ? make_float2(0.5f * (z1.y + z2.y), 0.5f * (z2.x - z1.x))
                           : make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y));
        dst[(size_t)l * half + mm] = o;
    }
}

// Index of kept output mode o (FFT order of an n-point axis) in an m-point FFT;
// -1 for the Nyquist slot.
__device__ __forceinline__ int kept_source(int o, int n, int m) {
    if (o == n / 2) return -1;
    int mo = o < n / 2 ? o : o - n;
    return (mo + m) & (m - 1);
}

// a2: y pass over [slab][z][y][mx] -> [slab][z][my][mx], m points pruned to n.
__global__ __launch_bounds__(kThreads) void k_fft_y(const float2* __restrict__ in, float2* __restrict__ out,
                                                    int m, int n, int half, int cols,
                                                    const float2* __restrict__ tw) {
    extern __shared__ float2 lds[];
    float2* a = lds;
    float2* b = lds + m * cols;
    const int c0 = blockIdx.x * cols;
    const size_t plane = (size_t)blockIdx.z * m + blockIdx.y;  // slab * m + z
    const float2* src = in + plane * m * half + c0;
    for (int t = threadIdx.x; t < m * cols; t += blockDim.x) {
        int i = t / cols, c = t % cols;
        a[i * cols + c] = src[(size_t)i * half + c];
    }
    __syncthreads();
    float2* res = fft_cols<-1>(a, b, cols, 1, m, cols, tw);
    float2* dst = out + plane * n * half + c0;
    for (int t = threadIdx.x; t < n * cols; t += blockDim.x) {
        int o = t / cols, c = t % cols;
        int src_i = kept_source(o, n, m);
        dst[(size_t)o * half + c] = src_i < 0 ? make_float2(0.f, 0.f) : res[src_i * cols + c];
    }
}

// Shared part of the z pass: transform each component's z-columns for one my
// row and accumulate sum_c vtab[c][|m|^2] * G_c into acc[mz][col].
__device__ void z_accumulate(const float2* __restrict__ in, int s, int q, int m, int n, int half, int cols,
                             int iy, int c0, const float* __restrict__ vtab, int m2n, float2* a, float2* b,
                             float2* acc, const float2* __restrict__ twm) {
    const int my = signed_mode(iy, n);
    for (int t = threadIdx.x; t < n * cols; t += blockDim.x) acc[t] = make_float2(0.f, 0.f);
    for (int c = 0; c < q; ++c) {
        const float2* src = in + (((size_t)s * q + c) * m) * n * half + (size_t)iy * half + c0;
        for (int t = threadIdx.x; t < m * cols; t += blockDim.x) {
            int i = t / cols, cc = t % cols;
            a[i * cols + cc] = src[(size_t)i * n * half + cc];
        }
        __syncthreads();
        float2* res = fft_cols<-1>(a, b, cols, 1, m, cols, twm);
        const float* vt = vtab + (size_t)c * m2n;
        for (int t = threadIdx.x; t < n * cols; t += blockDim.x) {
            int o = t / cols, cc = t % cols;
            int src_i = kept_source(o, n, m);
            if (src_i < 0) continue;
            int mz = signed_mode(o, n), mx = c0 + cc;
            float v = vt[mx * mx + my * my + mz * mz];
            float2 g = res[src_i * cols + cc];
            acc[t].x += v * g.x;
            acc[t].y += v * g.y;
        }
        __syncthreads();
    }
}

// a2 (z) + a3 for the fixed shape or a single spectrum: F = D(m) * acc.
__global__ __launch_bounds__(kThreads) void k_fft_z_spectrum(const float2* __restrict__ in, int q,
                                                             const float* __restrict__ vtab, int m2n,
                                                             const double* __restrict__ deconv,
                                                             float2* __restrict__ spec, int m, int n, int half,
                                                             int cols, const float2* __restrict__ twm) {
    extern __shared__ float2 lds[];
    float2* a = lds;
    float2* b = a + m * cols;
    float2* acc = b + m * cols;
    const int c0 = blockIdx.x * cols, iy = blockIdx.y, s = blockIdx.z;
    float2* dst = spec + (size_t)s * n * n * half + (size_t)iy * half + c0;
    if (iy == n / 2) {
        for (int t = threadIdx.x; t < n * cols; t += blockDim.x)
            dst[(size_t)(t / cols) * n * half + t % cols] = make_float2(0.f, 0.f);
        return;
    }
    z_accumulate(in, s, q, m, n, half, cols, iy, c0, vtab, m2n, a, b, acc, twm);
    for (int t = threadIdx.x; t < n * cols; t += blockDim.x) {
        int o = t / cols, cc = t % cols;
        float d = (float)(deconv[c0 + cc] * deconv[iy] * deconv[o]);
        dst[(size_t)o * n * half + cc] = make_float2(acc[t].x * d, acc[t].y * d);
    }
}

// a2 (z) + a3 + a4 + inverse z for the rotated shape:
//   S = F_A * conj(acc) * prod_d D(m_d) exp(i k_d o_d) / L   (FP64 factor),
// then the unnormalised inverse transform along z.
__global__ __launch_bounds__(kThreads) void k_fft_z_product(const float2* __restrict__ in, int q,
                                                            const float* __restrict__ vtab, int m2n,
                                                            const double2* __restrict__ phase,
                                                            const float2* __restrict__ fa, float2* __restrict__ out,
                                                            int m, int n, int half, int cols,
                                                            const float2* __restrict__ twm,
                                                            const float2* __restrict__ twn) {
    extern __shared__ float2 lds[];
    float2* a = lds;
    float2* b = a + m * cols;
    float2* acc = b + m * cols;
    const int c0 = blockIdx.x * cols, iy = blockIdx.y, s = blockIdx.z;
    float2* dst = out + (size_t)s * n * n * half + (size_t)iy * half + c0;
    if (iy == n / 2) {
        for (int t = threadIdx.x; t < n * cols; t += blockDim.x)
            dst[(size_t)(t / cols) * n * half + t % cols] = make_float2(0.f, 0.f);
        return;
    }
    z_accumulate(in, s, q, m, n, half, cols, iy, c0, vtab, m2n, a, b, acc, twm);
    const double2 py = phase[n + iy];
    for (int t = threadIdx.x; t < n * cols; t += blockDim.x) {
        int o = t / cols, cc = t % cols;
        double2 px = phase[c0 + cc], pz = phase[2 * n + o];
        // f = px * py * pz in FP64
        double fr = px.x * py.x - px.y * py.y, fi = px.x * py.y + px.y * py.x;
        double gr = fr * pz.x - fi * pz.y, gi = fr * pz.y + fi * pz.x;
        float2 fac = make_float2((float)gr, (float)gi);
        float2 A = fa[((size_t)o * n + iy) * half + c0 + cc];
        float2 cb = make_float2(acc[t].x, -acc[t].y);
        a[o * cols + cc] = cmul(cmul(A, cb), fac);
    }
    __syncthreads();
    float2* res = fft_cols<1>(a, b, cols, 1, n, cols, twn);
    for (int t = threadIdx.x; t < n * cols; t += blockDim.x) {
        int z = t / cols, cc = t % cols;
        dst[(size_t)z * n * half + cc] = res[z * cols + cc];
    }
}

// a5: inverse y over [s][z][my][mx] -> [s][z][y][mx].
__global__ __launch_bounds__(kThreads) void k_ifft_y(const float2* __restrict__ in, float2* __restrict__ out,
                                                     int n, int half, int cols, const float2* __restrict__ twn) {
    extern __shared__ float2 lds[];
    float2* a = lds;
    float2* b = lds + n * cols;
    const int c0 = blockIdx.x * cols;
    const size_t plane = (size_t)blockIdx.z * n + blockIdx.y;
    const float2* src = in + plane * n * half + c0;
    for (int t = threadIdx.x; t < n * cols; t += blockDim.x) {
        int i = t / cols, c = t % cols;
        a[i * cols + c] = src[(size_t)i * half + c];
    }
    __syncthreads();
    float2* res = fft_cols<1>(a, b, cols, 1, n, cols, twn);
    float2* dst = out + plane * n * half + c0;
    for (int t = threadIdx.x; t < n * cols; t += blockDim.x) {
        int i = t / cols, c = t % cols;
        dst[(size_t)i * half + c] = res[i * cols + c];
    }
}

// a5: inverse x, half-complex to real.  Two lines X1, X2 share one complex
// transform of Z = X1 + i X2 with both extended by Hermitian symmetry
// (X[n-m] = conj X[m], Nyquist 0, imaginary part of X[0] dropped); the real and
// imaginary parts of the result are the two score lines.  Each block also
// reduces its scores to (max, lowest index of the max).
__global__ __launch_bounds__(kThreads) void k_ifft_x(const float2* __restrict__ in, float* __restrict__ scores,
                                                     float* __restrict__ pval, int* __restrict__ pidx, int n,
                                                     int half, int cols, const float2* __restrict__ twn) {
    extern __shared__ float2 lds[];
    __shared__ float red_v[kThreads];
    __shared__ int red_i[kThreads];
    const int sc = n + 1;
    float2* a = lds;
    float2* b = lds + cols * sc;
    const int s = blockIdx.y;
    const size_t line0 = (size_t)blockIdx.x * 2 * cols;
    const float2* src = in + (size_t)s * n * n * half + line0 * half;
    for (int t = threadIdx.x; t < cols * n; t += blockDim.x) {
        int c = t / n, mm = t % n;
        float2 z;
        if (mm == half) {
            z = make_float2(0.f, 0.f);
        } else {
            bool lo = mm < half;
            int mi = lo ? mm : n - mm;
            float2 x1 = src[(size_t)(2 * c) * half + mi];
            float2 x2 = src[(size_t)(2 * c + 1) * half + mi];
            if (mi == 0) {
                x1.y = 0.f;
                x2.y = 0.f;
            }
            if (!lo) {
                x1.y = -x1.y;
                x2.y = -x2.y;
            }
            z = make_float2(x1.x - x2.y, x1.y + x2.x);
        }
        a[c * sc + mm] = z;
    }
    __syncthreads();
    float2* res = fft_cols<1>(a, b, 1, sc, n, cols, twn);
    float best = -INFINITY;
    int besti = 0x7fffffff;
    float* dst = scores ? scores + (size_t)s * n * n * n + line0 * n : nullptr;
    for (int t = threadIdx.x; t < 2 * cols * n; t += blockDim.x) {
        int l = t / n, x = t % n;
        float2 zz = res[(l >> 1) * sc + x];
        float v = (l & 1) ? zz.y : zz.x;
        if (dst) dst[(size_t)l * n + x] = v;
        int gi = (int)((line0 + l) * n + x);
        if (v > best || (v == best && gi < besti)) {
            best = v;
            besti = gi;
        }
    }
    red_v[threadIdx.x] = best;
    red_i[threadIdx.x] = besti;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            float v2 = red_v[threadIdx.x + off];
            int i2 = red_i[threadIdx.x + off];
            if (v2 > red_v[threadIdx.x] || (v2 == red_v[threadIdx.x] && i2 < red_i[threadIdx.x])) {
                red_v[threadIdx.x] = v2;
                red_i[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pval[(size_t)s * gridDim.x + blockIdx.x] = red_v[0];
        pidx[(size_t)s * gridDim.x + blockIdx.x] = red_i[0];
    }
}

__global__ __launch_bounds__(kThreads) void k_peak_final(const float* __restrict__ pval, const int* __restrict__ pidx,
                                                         int nblocks, float* __restrict__ out_val,
                                                         int64_t* __restrict__ out_idx) {
    __shared__ float red_v[kThreads];
    __shared__ int red_i[kThreads];
    const int s = blockIdx.x;
    float best = -INFINITY;
    int besti = 0x7fffffff;
    for (int t = threadIdx.x; t < nblocks; t += blockDim.x) {
        float v = pval[(size_t)s * nblocks + t];
        int i = pidx[(size_t)s * nblocks + t];
        if (v > best || (v == best && i < besti)) {
            best = v;
            besti = i;
        }
    }
    red_v[threadIdx.x] = best;
    red_i[threadIdx.x] = besti;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            float v2 = red_v[threadIdx.x + off];
            int i2 = red_i[threadIdx.x + off];
            if (v2 > red_v[threadIdx.x] || (v2 == red_v[threadIdx.x] && i2 < red_i[threadIdx.x])) {
                red_v[threadIdx.x] = v2;
                red_i[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out_val[s] = red_v[0];
        out_idx[s] = red_i[0];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_deconv_tables(const Geom& g, double box, const double origin[3], double* d_deconv,
                                double2* d_phase, hipStream_t st) {
    hipLaunchKernelGGL(k_deconv_tables, dim3((g.n + 127) / 128), dim3(128), 0, st, g.n, g.m, g.w,
                       (double)g.beta, box, origin[0], origin[1], origin[2], d_deconv, d_phase);
    return hipGetLastError();
}

hipError_t launch_ball_table(const Geom& g, double dk, const double* d_nodes, const double* d_basis, int p,
                             int q, double rhi, float* d_vtab, hipStream_t st) {
    hipLaunchKernelGGL(k_ball_table, dim3((g.m2n + 127) / 128), dim3(128), 0, st, g.m2n, dk, d_nodes, d_basis,
                       p, q, rhi, d_vtab);
    return hipGetLastError();
}

hipError_t launch_rotate(const Geom& g, const double* d_quats, int S, const double* d_pos, int64_t nk,
                         float4* d_knots, hipStream_t st) {
    if (nk == 0 || S == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rotate, dim3((unsigned)((nk + 255) / 256), S), dim3(256), 0, st, d_quats, d_pos, nk,
                       g.inv_hf, g.m, d_knots);
    return hipGetLastError();
}

hipError_t launch_zero(float* p, size_t count, hipStream_t st) {
    size_t n4 = count / 4;  // all buffers are multiples of 4 floats
    if (n4 == 0) return hipSuccess;
    size_t blocks = (n4 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<float4*>(p), n4);
    return hipGetLastError();
}

hipError_t launch_spread(const Geom& g, const float4* d_knots, int S, int64_t nk, const float* d_wts, int q,
                         float* d_fine, hipStream_t st) {
    if (nk == 0 || S == 0) return hipSuccess;
    hipLaunchKernelGGL(k_spread, dim3((unsigned)nk, S), dim3(64), 0, st, d_knots, nk, d_wts, q, g.m, g.w, g.beta,
                       g.inv_i0beta, d_fine);
    return hipGetLastError();
}

hipError_t launch_fft_x(const Geom& g, const float* d_fine, int slabs, float2* d_out, const float2* d_twm,
                        hipStream_t st) {
    const int cols = fft_cols_for(g.m, g.m * g.m / 2);
    const size_t lds = sizeof(float2) * 2 * (size_t)cols * (g.m + 1);
    hipLaunchKernelGGL(k_fft_x, dim3((unsigned)(g.m * g.m / (2 * cols)), slabs), dim3(kThreads), lds, st, d_fine,
                       d_out, g.m, g.half, cols, d_twm);
    return hipGetLastError();
}

hipError_t launch_fft_y(const Geom& g, const float2* d_in, int slabs, float2* d_out, const float2* d_twm,
                        hipStream_t st) {
    const int cols = fft_cols_for(g.m, g.half);
    const size_t lds = sizeof(float2) * 2 * (size_t)cols * g.m;
    hipLaunchKernelGGL(k_fft_y, dim3(g.half / cols, g.m, slabs), dim3(kThreads), lds, st, d_in, d_out, g.m, g.n,
                       g.half, cols, d_twm);
    return hipGetLastError();
}

hipError_t launch_fft_z_spectrum(const Geom& g, const float2* d_in, int S, int q, const float* d_vtab,
                                 const double* d_deconv, float2* d_spec, const float2* d_twm, hipStream_t st) {
    const int cols = fft_cols_for(g.m, g.half);
    const size_t lds = sizeof(float2) * ((size_t)2 * cols * g.m + (size_t)cols * g.n);
    hipLaunchKernelGGL(k_fft_z_spectrum, dim3(g.half / cols, g.n, S), dim3(kThreads), lds, st, d_in, q, d_vtab,
                       g.m2n, d_deconv, d_spec, g.m, g.n, g.half, cols, d_twm);
    return hipGetLastError();
}

hipError_t launch_fft_z_product(const Geom& g, const float2* d_in, int S, int q, const float* d_vtab,
                                const double2* d_phase, const float2* d_fa, float2* d_out, const float2* d_twm,
                                const float2* d_twn, hipStream_t st) {
    const int cols = fft_cols_for(g.m, g.half);
    const size_t lds = sizeof(float2) * ((size_t)2 * cols * g.m + (size_t)cols * g.n);
    hipLaunchKernelGGL(k_fft_z_product, dim3(g.half / cols, g.n, S), dim3(kThreads), lds, st, d_in, q, d_vtab,
                       g.m2n, d_phase, d_fa, d_out, g.m, g.n, g.half, cols, d_twm, d_twn);
    return hipGetLastError();
}

hipError_t launch_ifft_y(const Geom& g, const float2* d_in, int S, float2* d_out, const float2* d_twn,
                         hipStream_t st) {
    const int cols = fft_cols_for(g.n, g.half);
    const size_t lds = sizeof(float2) * 2 * (size_t)cols * g.n;
    hipLaunchKernelGGL(k_ifft_y, dim3(g.half / cols, g.n, S), dim3(kThreads), lds, st, d_in, d_out, g.n, g.half,
                       cols, d_twn);
    return hipGetLastError();
}

int ifft_x_blocks(const Geom& g) {
    const int cols = fft_cols_for(g.n, g.n * g.n / 2);
    return g.n * g.n / (2 * cols);
}

hipError_t launch_ifft_x(const Geom& g, const float2* d_in, int S, float* d_scores, float* d_pval, int* d_pidx,
                         const float2* d_twn, hipStream_t st) {
    const int cols = fft_cols_for(g.n, g.n * g.n / 2);
    const size_t lds = sizeof(float2) * 2 * (size_t)cols * (g.n + 1);
    hipLaunchKernelGGL(k_ifft_x, dim3((unsigned)ifft_x_blocks(g), S), dim3(kThreads), lds, st, d_in, d_scores,
                       d_pval, d_pidx, g.n, g.half, cols, d_twn);
    return hipGetLastError();
}

hipError_t launch_peak_final(const float* d_pval, const int* d_pidx, int S, int nblocks, float* d_peak_val,
                             int64_t* d_peak_idx, hipStream_t st) {
    hipLaunchKernelGGL(k_peak_final, dim3(S), dim3(kThreads), 0, st, d_pval, d_pidx, nblocks, d_peak_val,
                       d_peak_idx);
    return hipGetLastError();
}

}  // namespace corr

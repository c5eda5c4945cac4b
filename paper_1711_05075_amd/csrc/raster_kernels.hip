// gfx950 kernels of the uniform-rasterization baseline (Behandish & Ilies,
// Sec. 5.2 and Sec. 6.2: sample both shapes on a uniform grid, correlate the
// two grids by FFT: two forward transforms, a pointwise product, one inverse).
//
// The fixed shape is sampled at origin + h u and the moved shape (turned by R)
// at h v, u, v in [0, n)^3 with v read as a signed index (v - n for v >= n/2),
// a sample being 1 when it lies in some ball: |p - c|^2 <= r^2 in FP64.  The
// count at translation index t is sum_u a(u) b(u - t) over periodic indices:
// the samples where the fixed shape meets the moved one translated by
// origin + h t.  Both grids go into one complex grid a + i b, whose FP64
// transform Z gives A(k) = (Z_k + conj Z_-k) / 2 and B(k) = (Z_k - conj Z_-k) / 2i;
// the inverse transform of A conj(B) is n^3 times the counts, which FP64 holds
// to far better than 1/2, so they are rounded to exact integers.
#include "corr_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

namespace corr {
namespace {

constexpr int kRThreads = 256;

__global__ __launch_bounds__(kRThreads) void k_zero2(double2* __restrict__ p, size_t count) {
    for (size_t i = (size_t)blockIdx.x * kRThreads + threadIdx.x; i < count; i += (size_t)gridDim.x * kRThreads)
        p[i] = make_double2(0.0, 0.0);
}

// One workgroup per ball: every sample of the ball's bounding box (one sample
// of margin on each side) that lies in the ball gets 1 in the real part (the
// fixed shape, which = 0) or the imaginary part (the moved shape, which = 1,
// turned by the unit quaternion quat).  Several balls may mark one sample;
// they all store the same value.
__global__ __launch_bounds__(kRThreads) void k_raster(const double* __restrict__ pos, const double* __restrict__ rad,
                                                      const double* __restrict__ quat, double o0, double o1, double o2,
                                                      double h, int n, int which, double2* __restrict__ grid) {
    const int64_t j = blockIdx.x;
    double c[3] = {pos[3 * j], pos[3 * j + 1], pos[3 * j + 2]};
    if (which == 1) {
        const double* q = quat;
        const double nn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const double w = q[0] / nn, x = q[1] / nn, y = q[2] / nn, z = q[3] / nn;
        const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),    2 * (x * z + w * y),
                             2 * (x * y + w * z),    1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                             2 * (x * z - w * y),    2 * (y * z + w * x),    1 - 2 * (x * x + y * y)};
        const double p0 = c[0], p1 = c[1], p2 = c[2];
        c[0] = R[0] * p0 + R[1] * p1 + R[2] * p2;
        c[1] = R[3] * p0 + R[4] * p1 + R[5] * p2;
        c[2] = R[6] * p0 + R[7] * p1 + R[8] * p2;
    }
    const double r = rad[j], r2 = r * r;
    const double org[3] = {which ? 0.0 : o0, which ? 0.0 : o1, which ? 0.0 : o2};
    // sample index range per axis: the fixed grid's u in [0, n), the moved
    // grid's signed v in [-n/2, n/2)
    const int lo_all = which ? -n / 2 : 0, hi_all = which ? n / 2 - 1 : n - 1;
    int lo[3], ext[3];
    for (int d = 0; d < 3; ++d) {
        const double f = (c[d] - org[d]) / h, s = r / h;
        const double a = floor(f - s) - 1.0, b = floor(f + s) + 1.0;
        const int l = (int)fmax(a, (double)lo_all), u = (int)fmin(b, (double)hi_all);
        lo[d] = l;
        ext[d] = u >= l ? u - l + 1 : 0;
    }
    const int cells = ext[0] * ext[1] * ext[2];
    for (int t = threadIdx.x; t < cells; t += kRThreads) {
        const int ix = lo[0] + t % ext[0], iy = lo[1] + (t / ext[0]) % ext[1], iz = lo[2] + t / (ext[0] * ext[1]);
        double p[3];
        if (which) {
            p[0] = h * ix;
            p[1] = h * iy;
            p[2] = h * iz;
        } else {
            p[0] = o0 + h * ix;
            p[1] = o1 + h * iy;
            p[2] = o2 + h * iz;
        }
        const double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
        if (dx * dx + dy * dy + dz * dz <= r2) {
            const size_t k = ((size_t)((iz + n) % n) * n + (iy + n) % n) * n + (ix + n) % n;
            if (which) grid[k].y = 1.0;
            else grid[k].x = 1.0;
        }
    }
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}

// Unnormalised FP64 DFT along one axis of an n^3 grid ([z][y][x]), sum_j
// x_j exp(SIGN 2 pi i j s / N), for COLS lines per workgroup, as radix-2
// Stockham autosort passes in LDS.  Lines of axis 0 are contiguous; those of
// axes 1 and 2 are taken COLS adjacent x at a time, so that every access is a
// row segment.  tw[j] = exp(-2 pi i j / N).
template <int N, int COLS>
__global__ __launch_bounds__(kRThreads) void k_fft64(double2* __restrict__ data, int axis, int sign,
                                                     const double2* __restrict__ tw) {
    __shared__ double2 a[COLS * N];
    __shared__ double2 twl[N];
    double2* cube = data + (size_t)blockIdx.y * N * N * N;
    const size_t stride = axis == 0 ? 1 : axis == 1 ? (size_t)N : (size_t)N * N;
    const int l0 = blockIdx.x * COLS;
    auto base = [&](int l) -> size_t {
        if (axis == 0) return (size_t)l * N;  // l = z N + y
        if (axis == 1) return (size_t)(l / N) * N * N + (l % N);  // l = z N + x
        return (size_t)l;  // axis 2: l = y N + x
    };
    for (int t = threadIdx.x; t < N; t += kRThreads) twl[t] = tw[t];
    // element (c, j) of the batch at a[c * N + j]
    for (int t = threadIdx.x; t < COLS * N; t += kRThreads) {
        const int c = axis == 0 ? t / N : t % COLS, j = axis == 0 ? t % N : t / COLS;
        a[c * N + j] = cube[base(l0 + c) + (size_t)j * stride];
    }
    __syncthreads();
    constexpr int NBF = (COLS * N / 2 + kRThreads - 1) / kRThreads;
    for (int ns = 1; ns < N; ns <<= 1) {
        double2 u[NBF], v[NBF];
        int oi[NBF];
#pragma unroll
        for (int b = 0; b < NBF; ++b) {
            const int t = b * kRThreads + threadIdx.x;
            if (t < COLS * N / 2) {
                const int c = t / (N / 2), j = t % (N / 2), k = j % ns;
                u[b] = a[c * N + j];
                double2 w = twl[k * (N / (2 * ns))];
                if (sign > 0) w.y = -w.y;
                v[b] = zmul(a[c * N + j + N / 2], w);
                oi[b] = c * N + (j / ns) * 2 * ns + k;
            }
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NBF; ++b) {
            const int t = b * kRThreads + threadIdx.x;
            if (t < COLS * N / 2) {
                a[oi[b]] = make_double2(u[b].x + v[b].x, u[b].y + v[b].y);
                a[oi[b] + ns] = make_double2(u[b].x - v[b].x, u[b].y - v[b].y);
            }
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < COLS * N; t += kRThreads) {
        const int c = axis == 0 ? t / N : t % COLS, j = axis == 0 ? t % N : t / COLS;
        cube[base(l0 + c) + (size_t)j * stride] = a[c * N + j];
    }
}

// Z -> A conj(B) with A = (Z_k + conj Z_-k) / 2, B = (Z_k - conj Z_-k) / 2i;
// each pair (k, -k) is handled by one thread, which writes both (the product
// of two real grids' transforms is Hermitian).
__global__ __launch_bounds__(kRThreads) void k_raster_product(double2* __restrict__ data, int n) {
    double2* cube = data + (size_t)blockIdx.y * n * n * n;
    const size_t n3 = (size_t)n * n * n;
    const size_t i = (size_t)blockIdx.x * kRThreads + threadIdx.x;
    if (i >= n3) return;
    const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((size_t)n * n));
    const size_t ni = ((size_t)((n - z) % n) * n + (n - y) % n) * n + (n - x) % n;
    if (ni < i) return;
    const double2 zk = cube[i], zm = cube[ni];
    const double2 A = make_double2(0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y));
    const double2 B = make_double2(0.5 * (zk.y + zm.y), 0.5 * (zm.x - zk.x));
    const double2 P = make_double2(fma(A.x, B.x, A.y * B.y), fma(A.y, B.x, -(A.x * B.y)));
    cube[i] = P;
    if (ni != i) cube[ni] = make_double2(P.x, -P.y);
}

// counts = round(re / n^3) after the unnormalised inverse transform.
__global__ __launch_bounds__(kRThreads) void k_raster_counts(const double2* __restrict__ data, int n,
                                                             int32_t* __restrict__ counts) {
    const size_t n3 = (size_t)n * n * n;
    const size_t i = (size_t)blockIdx.x * kRThreads + threadIdx.x;
    if (i < n3) counts[i] = (int32_t)llrint(data[i].x / (double)n3);
}

template <class F>
hipError_t with_n(int n, F&& f) {
    switch (n) {
        case 16: f(std::integral_constant<int, 16>{}); break;
        case 32: f(std::integral_constant<int, 32>{}); break;
        case 64: f(std::integral_constant<int, 64>{}); break;
        case 128: f(std::integral_constant<int, 128>{}); break;
        case 256: f(std::integral_constant<int, 256>{}); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_raster_counts(int n, double h, const double origin[3], const double* d_pos_a, const double* d_rad_a,
                                int64_t na, const double* d_pos_b, const double* d_rad_b, int64_t nb,
                                const double* d_quat, const double2* d_tw, double2* d_grid, int32_t* d_counts,
                                hipStream_t st) {
    const size_t n3 = (size_t)n * n * n;
    hipLaunchKernelGGL(k_zero2, dim3((unsigned)std::min<size_t>((n3 + kRThreads - 1) / kRThreads, 4096)),
                       dim3(kRThreads), 0, st, d_grid, n3);
    if (na > 0)
        hipLaunchKernelGGL(k_raster, dim3((unsigned)na), dim3(kRThreads), 0, st, d_pos_a, d_rad_a, d_quat, origin[0],
                           origin[1], origin[2], h, n, 0, d_grid);
    if (nb > 0)
        hipLaunchKernelGGL(k_raster, dim3((unsigned)nb), dim3(kRThreads), 0, st, d_pos_b, d_rad_b, d_quat, origin[0],
                           origin[1], origin[2], h, n, 1, d_grid);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = with_n(n, [&](auto nc) {
        constexpr int N = decltype(nc)::value;
        constexpr int COLS = N >= 128 ? 2048 / N : 16;
        for (int pass = 0; pass < 6; ++pass) {
            const int axis = pass % 3, sign = pass < 3 ? -1 : 1;
            if (pass == 3)
                hipLaunchKernelGGL(k_raster_product, dim3((unsigned)((n3 + kRThreads - 1) / kRThreads)),
                                   dim3(kRThreads), 0, st, d_grid, n);
            hipLaunchKernelGGL((k_fft64<N, COLS>), dim3(N * N / COLS), dim3(kRThreads), 0, st, d_grid, axis, sign,
                               d_tw);
        }
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_raster_counts, dim3((unsigned)((n3 + kRThreads - 1) / kRThreads)), dim3(kRThreads), 0, st,
                       d_grid, n, d_counts);
    return hipGetLastError();
}

}  // namespace corr

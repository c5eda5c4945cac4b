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
// thread does whole radix-R butterflies per pass in registers), over a batch of
// columns so that every HBM access is a contiguous row segment.  Kernels are
// templates on the spreading-grid size M (translation grid N = M/2), so every
// index computation is a shift or mask.
#include "corr_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace corr {
namespace {

constexpr int kThreads = 256;

// Workgroups go to the XCDs in turn (linear id mod kXcds), each XCD with an L2
// of its own.  xcd_block gives a workgroup its logical block (x fastest) so
// that the gridDim.x blocks of one (y, z) -- neighbouring column blocks, which
// read the two halves of the same 128-byte lines -- run one after another on
// one XCD and share its L2, while successive (y, z) go to the XCDs in turn,
// which keeps the XCDs evenly loaded.  A bijection of the grid onto itself
// (a tail of fewer than kXcds whole rows keeps the plain order): every
// block's work is unchanged.
constexpr int kXcds = 8;
struct Blk {
    int x, y, z;
};
__device__ __forceinline__ Blk xcd_block() {
    const int gx = (int)gridDim.x, gy = (int)gridDim.y;
    const int total = gx * gy * (int)gridDim.z;
    const int lin = (int)blockIdx.x + gx * ((int)blockIdx.y + gy * (int)blockIdx.z);
    const int span = kXcds * gx, main = total - total % span;
    int lam = lin;
    if (lin < main) {
        const int xcd = lin % kXcds, r = lin / kXcds;  // r-th workgroup of this XCD
        lam = ((r / gx) * kXcds + xcd) * gx + r % gx;
    }
    return {lam % gx, (lam / gx) % gy, lam / (gx * gy)};
}

// This file is built without floating-point contraction: every fused
// multiply-add is written out (fmaf), so the arithmetic and its rounding are
// fixed by the source and do not depend on how a kernel is instantiated
// (column batch, launch shape) or scheduled.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
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

// ---------------------------------------------------------------------------
// Column FFT engine.  A workgroup transforms COLS columns of LEN points held in
// LDS; element (i, c) lives at buf[i * SI + c * SC] ("LINES" layout: each
// column contiguous with a padded stride, otherwise columns interleaved).  The
// transform is a sequence of Stockham autosort passes of radix 8 (then 4 or 2)
// done in place: in every pass each thread first reads the inputs of all its
// butterflies into registers, the workgroup synchronises, and the outputs are
// written back over the same buffer.  All sizes are compile-time powers of
// two.  tw[j] = exp(-2 pi i j / LEN) is an LDS table.  With HALF only the
// outputs of index < LEN/4 or >= 3 LEN/4 are written by the last pass (the
// band the forward passes keep); the others are left unspecified, and the
// arithmetic that only they need is not done.
// ---------------------------------------------------------------------------
template <int LEN, int NS, int SIGN, int COLS, int SI, int SC, int NT, bool HALF = false>
__device__ __forceinline__ void fft_passes(float2* a, const float2* tw) {
    if constexpr (NS < LEN) {
        constexpr int REM = LEN / NS;
        constexpr int R = REM >= 8 ? 8 : REM;
        constexpr int NB = LEN / R;
        constexpr int TWS = LEN / (NS * R);
        constexpr int WORK = NB * COLS;
        constexpr int NBF = (WORK + NT - 1) / NT;
        float2 v[NBF][R];
#pragma unroll
        for (int u = 0; u < NBF; ++u) {
            const int t = u * NT + (int)threadIdx.x;
            if (WORK % NT == 0 || t < WORK) {
                const int c = t % COLS, j = t / COLS;
                const int k = j % NS;
#pragma unroll
                for (int r = 0; r < R; ++r) v[u][r] = a[(j + r * NB) * SI + c * SC];
                if constexpr (NS > 1) {
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        float2 w = tw[r * k * TWS];
                        if constexpr (SIGN > 0) w.y = -w.y;
                        v[u][r] = cmul(v[u][r], w);
                    }
                }
                if constexpr (R == 8) dft8<SIGN>(v[u]);
                else if constexpr (R == 4) dft4<SIGN>(v[u][0], v[u][1], v[u][2], v[u][3]);
                else dft2<SIGN>(v[u]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NBF; ++u) {
            const int t = u * NT + (int)threadIdx.x;
            if (WORK % NT == 0 || t < WORK) {
                const int c = t % COLS, j = t / COLS;
                const int k = j % NS;
                const int o = (j / NS) * NS * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // last pass: output k + r LEN/R (k < LEN/R) is in the band iff
                    // r < R/4 or r >= 3R/4 (R = 4, 8); for R = 2 it depends on k
                    if constexpr (HALF && NS * R == LEN) {
                        if constexpr (R >= 4) {
                            if (r >= R / 4 && r < 3 * R / 4) continue;
                        } else {
                            if ((r == 0) != (k < LEN / 4)) continue;
                        }
                    }
                    a[(o + r * NS) * SI + c * SC] = v[u][r];
                }
            }
        }
        __syncthreads();
        fft_passes<LEN, NS * R, SIGN, COLS, SI, SC, NT, HALF>(a, tw);
    }
}

// Unnormalised DFT sum_i x_i exp(SIGN 2 pi i i s / LEN) of every column, in
// place, by a workgroup of NT threads.  Entered by the whole workgroup once the
// input in `a` and the table are visible; the result is visible to the whole
// workgroup on return.
template <int LEN, int SIGN, int COLS, bool LINES, int NT = kThreads>
__device__ __forceinline__ void fft_cols(float2* a, const float2* tw) {
    fft_passes<LEN, 1, SIGN, COLS, (LINES ? 1 : COLS), (LINES ? LEN + 1 : 1), NT>(a, tw);
}

template <int LEN, int NT = kThreads>
__device__ __forceinline__ void load_table(float2* dst, const float2* __restrict__ src) {
    for (int t = threadIdx.x; t < LEN; t += NT) dst[t] = src[t];
}

template <int A, int B>
constexpr int cmin() { return A < B ? A : B; }

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

// vtab[c][m2] = (4 pi / 3) rref^3 sum_b f(k, r_b) basis[b][c], k = dk sqrt(m2): the
// k-factor of the separable radius expansion of the per-ball kernel
//   K(k; r) = Bhat(k; r + r0) - lam Bhat(k; r) = (4 pi / 3) rref^3 f(k, r),
//   f(k, r) = ((r + r0) / rref)^3 Phi(k (r + r0)) - lam (r / rref)^3 Phi(k r).
// The overlap score is r0 = lam = 0 (the ball transform itself); the
// shape-complementarity affinity (Sec. 4.2) has r0, lam > 0.
__global__ void k_ball_table(int m2n, double dk, const double* __restrict__ nodes,
                             const double* __restrict__ basis, int p, int q, double rref, double r0,
                             double lam, float* __restrict__ vtab) {
    int m2 = blockIdx.x * blockDim.x + threadIdx.x;
    if (m2 >= m2n) return;
    double k = dk * sqrt((double)m2);
    double acc[32];
    for (int c = 0; c < q; ++c) acc[c] = 0.0;
    for (int b = 0; b < p; ++b) {
        const double rg = (nodes[b] + r0) / rref, rr = nodes[b] / rref;
        double f = rg * rg * rg * ball_shape(k * (nodes[b] + r0));
        if (lam != 0.0) f -= lam * rr * rr * rr * ball_shape(k * nodes[b]);
        for (int c = 0; c < q; ++c) acc[c] += f * basis[b * q + c];
    }
    double scale = 4.0 * M_PI / 3.0 * rref * rref * rref;
    for (int c = 0; c < q; ++c) vtab[(size_t)c * m2n + m2] = (float)(scale * acc[c]);
}

// 3D Fourier transform at |k| of the 4D volume W(|t|; P) = pi (P^2 - |t|^2)^2 / 24
// of the intersection of two opposite cones (the lifted kernel of Sec. 3.1,
// eq. eq_convgA, sliced at one height), whose cross-sections' radii sum to P:
//   What(k; P) = 4 pi^2 (x^3 cos x - 6 x^2 sin x - 15 x cos x + 15 sin x) / (3 k^7),
// x = k P; below x = 2 the closed form cancels to x^7 and its Taylor series
// P^7 (4 pi^2 / 3) sum_n (-1)^n (2n+2)(2n+4)(2n+6) x^(2n) / (2n+7)! is summed
// (18 terms leave < 1e-17 relative at x = 2).  Zero for P <= 0.
__device__ double lift_what(double k, double P) {
    if (!(P > 0.0)) return 0.0;
    const double x = k * P;
    if (x < 2.0) {
        const double x2 = x * x;
        double term = 1.0, sum = 0.0, fact = 5040.0;
        for (int n = 0; n < 18; ++n) {
            const double c = (2.0 * n + 2) * (2.0 * n + 4) * (2.0 * n + 6) / fact;
            sum += ((n & 1) ? -c : c) * term;
            term *= x2;
            fact *= (2.0 * n + 8) * (2.0 * n + 9);
        }
        const double p2 = P * P;
        return 4.0 * M_PI * M_PI / 3.0 * p2 * p2 * p2 * P * sum;
    }
    double sn, cs;
    sincos(x, &sn, &cs);
    const double k2 = k * k, k7 = k2 * k2 * k2 * k;
    return 4.0 * M_PI * M_PI * (x * x * x * cs - 6.0 * x * x * sn - 15.0 * x * cs + 15.0 * sn) / (3.0 * k7);
}

// tab[p][p'][m2] = What(dk sqrt(m2); a_p + b_p' - h): the lifted kernel at the
// radius nodes of both shapes for one slice height h, the bilinear expansion
//   What(k; r_i + rho_j - h) ~ sum_{p,p'} l_p(r_i) l'_p'(rho_j) tab[p][p'](k).
__global__ void k_lift_table(int m2n, double dk, const double* __restrict__ na, int qa,
                             const double* __restrict__ nb, int qb, double h, float* __restrict__ tab) {
    const int m2 = blockIdx.x * blockDim.x + threadIdx.x;
    const int pp = blockIdx.y;  // p * qb + p'
    if (m2 >= m2n) return;
    const int p = pp / qb, p2 = pp % qb;
    tab[(size_t)pp * m2n + m2] = (float)lift_what(dk * sqrt((double)m2), na[p] + nb[p2] - h);
}

// ---------------------------------------------------------------------------
// a0 (binned form): rotate + place + window weights, and a counting sort of the
// knots by key = z-cell * nyb + y-cell / ygroup, so that a spreading tile finds
// the knots that reach it as a few short ranges of the sorted order.  Ranks come
// from atomic counters, so equal keys are ordered by scheduling: every later
// sum over knots is exact integer arithmetic, so results do not depend on it.
// The counters are zero on entry and are cleared again by the scan.
// ---------------------------------------------------------------------------
constexpr int kBinBlock = 256;

// Exclusive scan of the per-thread values v over a kBinBlock-thread block;
// returns the sum over lower threads.
__device__ __forceinline__ int block_exclusive_scan(int v, int* wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(incl, d, 64);
        if (lane >= d) incl += u;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    return before + incl - v;
}

// Key starts from the counts of one rotation, PER consecutive keys per thread
// of a kBinBlock-thread block; clears the counts.
template <int PER>
__device__ __forceinline__ void scan_counts(int* __restrict__ cs, int* __restrict__ bs, int* wsum) {
    static_assert(PER % 4 == 0, "whole int4 per thread");
    const int b0 = threadIdx.x * PER;
    int v[PER];
#pragma unroll
    for (int k = 0; k < PER / 4; ++k) {
        const int4 x = reinterpret_cast<const int4*>(cs + b0)[k];
        v[4 * k] = x.x; v[4 * k + 1] = x.y; v[4 * k + 2] = x.z; v[4 * k + 3] = x.w;
    }
    int sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) sum += v[k];
    int run = block_exclusive_scan(sum, wsum);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int c = v[k];
        v[k] = run;
        run += c;
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) bs[b0 + k] = v[k];  // bs rows are keys + 1 long: not 16-byte aligned
#pragma unroll
    for (int k = 0; k < PER / 4; ++k) reinterpret_cast<int4*>(cs + b0)[k] = make_int4(0, 0, 0, 0);
}

// Rotate + place + counts per key: each knot's record is its packed cell and
// its offsets from that cell along x, y and z (FP32, in [0, 1)), from which the
// scatter evaluates the window weights.  Workgroup (0, 0) also clears the tile
// plan's counters.  The rank of a knot within its key depends on the order
// of the increments; the spreading sums do not (they are exact integers).
__global__ __launch_bounds__(kBinBlock) void k_rotate_bin(const double* __restrict__ quats,
                                                          const double* __restrict__ pos, int64_t nk, double inv_hf,
                                                          int m, int yshift, int nyb, int kstride,
                                                          int4* __restrict__ rec, int* __restrict__ rank,
                                                          int* __restrict__ counts, int* __restrict__ plan,
                                                          int nplan) {
    const int64_t j = (int64_t)blockIdx.x * kBinBlock + threadIdx.x;
    const int s = blockIdx.y;
    if (blockIdx.x == 0 && s == 0 && (int)threadIdx.x < nplan) plan[threadIdx.x] = 0;
    int key = -1;
    if (j < nk) {
        const double* q = quats + 4 * s;
        double nn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        double qw = q[0] / nn, x = q[1] / nn, y = q[2] / nn, z = q[3] / nn;
        double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - qw * z),    2 * (x * z + qw * y),
                       2 * (x * y + qw * z),    1 - 2 * (x * x + z * z), 2 * (y * z - qw * x),
                       2 * (x * z - qw * y),    2 * (y * z + qw * x),    1 - 2 * (x * x + y * y)};
        double px = pos[3 * j], py = pos[3 * j + 1], pz = pos[3 * j + 2];
        double u[3] = {(R[0] * px + R[1] * py + R[2] * pz) * inv_hf, (R[3] * px + R[4] * py + R[5] * pz) * inv_hf,
                       (R[6] * px + R[7] * py + R[8] * pz) * inv_hf};
        int c[3];
        float f3[3];
        for (int d = 0; d < 3; ++d) {
            double fl = floor(u[d]);
            float f = (float)(u[d] - fl);
            c[d] = (int)((long long)fl & (long long)(m - 1));  // m is a power of two
            if (f >= 1.0f) {
                f = 0.0f;
                c[d] = (c[d] + 1) & (m - 1);
            }
            f3[d] = f;
        }
        rec[(int64_t)s * nk + j] = make_int4(c[0] | (c[1] << 10) | (c[2] << 20), __float_as_int(f3[0]),
                                             __float_as_int(f3[1]), __float_as_int(f3[2]));
        key = c[2] * nyb + (c[1] >> yshift);
    }
    // the lanes of a wave that share a key take one counter increment: the
    // lowest of them adds the group's size, and each gets the base plus its
    // place among the group's lanes.  Every lane runs the loop (one pass per
    // distinct key of the wave); lanes past nk have no key.
    const int lane = threadIdx.x & 63;
    int* cnt = counts + (size_t)s * kstride;
    unsigned long long todo = __ballot(key >= 0), same = 0;
    while (todo) {
        const int lk = __builtin_amdgcn_readlane(key, __ffsll(todo) - 1);
        const unsigned long long grp = __ballot(key == lk);
        if (key == lk) same = grp;
        todo &= ~grp;
    }
    const int first = same ? __ffsll(same) - 1 : lane;
    int base = 0;
    if (key >= 0 && first == lane) base = atomicAdd(cnt + key, __popcll(same));
    base = __shfl(base, first, 64);
    if (j < nk) rank[(int64_t)s * nk + j] = base + __popcll(same & ((1ull << lane) - 1ull));
}

// Key starts of each rotation from its counts (one workgroup per rotation,
// keys / kBinBlock consecutive keys per thread); clears the counts.  Reading
// the counts in a kernel of its own makes every workgroup's atomic increments
// visible without device-wide fences.
__global__ __launch_bounds__(kBinBlock) void k_bin_scan(int* __restrict__ counts, int keys, int kstride,
                                                        int64_t nk, int* __restrict__ bin_start) {
    __shared__ int wsum[kBinBlock / 64];
    const int s = blockIdx.x;
    int* cs = counts + (size_t)s * kstride;
    int* bs = bin_start + (size_t)s * (kstride + 1);
    switch (keys / kBinBlock) {  // keys is a power of two, 1024 .. 32768
        case 4: scan_counts<4>(cs, bs, wsum); break;
        case 8: scan_counts<8>(cs, bs, wsum); break;
        case 16: scan_counts<16>(cs, bs, wsum); break;
        case 32: scan_counts<32>(cs, bs, wsum); break;
        case 64: scan_counts<64>(cs, bs, wsum); break;
        default: scan_counts<128>(cs, bs, wsum); break;
    }
    if (threadIdx.x == 0) bs[keys] = (int)nk;
}

// Scatter knot j of rotation s into sorted position: its packed cell, its
// window weights along x, y and z (evaluated here from its offsets, w per
// axis) and its q component weights.
__device__ __forceinline__ void bin_scatter(int64_t j, int s, const int4* __restrict__ rec,
                                            const float* __restrict__ wts, const int* __restrict__ rank,
                                            const int* __restrict__ bin_start, int64_t nk, int keys, int yshift,
                                            int nyb, int w, float beta, float inv_i0beta, int q,
                                            int* __restrict__ scell, float* __restrict__ skbw,
                                            float* __restrict__ swts) {
    const int4 r = rec[(int64_t)s * nk + j];
    const int packed = r.x;
    const int key = ((packed >> 20) & 1023) * nyb + (((packed >> 10) & 1023) >> yshift);
    const int64_t p = (int64_t)s * nk + bin_start[(size_t)s * (keys + 1) + key] + rank[(int64_t)s * nk + j];
    scell[p] = packed;
    const float tw = 2.0f / (float)w;
    const int lo = w / 2 - 1;
    const float f3[3] = {__int_as_float(r.y), __int_as_float(r.z), __int_as_float(r.w)};
    float2* dst = reinterpret_cast<float2*>(skbw + p * 3 * w);
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < w; i += 2)
            dst[(d * w + i) / 2] = make_float2(kb_window(f3[d] - (float)(i - lo), tw, beta, inv_i0beta),
                                               kb_window(f3[d] - (float)(i + 1 - lo), tw, beta, inv_i0beta));
    for (int c = 0; c < q; ++c) swts[p * q + c] = wts[(size_t)c * nk + j];
}

// ---------------------------------------------------------------------------
// a1 + a2 (x): spreading fused with the x transform.  A workgroup owns TY full
// x-lines (z row z0, y rows y0 .. y0+TY-1).  For each pair of radius components
// (c, c+1) it accumulates both into one complex line (c in the real part, c+1
// in the imaginary part), transforms the lines along x in LDS and separates the
// two half spectra:
//   X_c = (Z_m + conj Z_{M-m}) / 2,  X_{c+1} = (Z_m - conj Z_{M-m}) / 2i.
// The knots that can reach the tile are those of the z-cells z0-w/2 ..
// z0+w/2-1 and of the y-groups that hold y-cells y0-w/2 .. y0+TY+w/2-2: at
// most two key ranges per z-cell of the sorted order.  Those whose window
// reaches the tile's rows are compacted in order (wave ballots + a block scan)
// and staged in LDS with their window weights; the component weights of each
// pair are then read by sorted position.  Each wave applies staged knots, a
// lane per window point, adding into 64-bit fixed-point sums with LDS integer
// atomics: integer addition is exact and associative, so the result does not
// depend on scheduling.  The fixed-point scale is a power of two chosen per
// shape so that every addend fits 32 bits (one conversion instruction) and no
// sum can overflow.  A tile that no knot reaches only records that in
// tile_live.
// ---------------------------------------------------------------------------
// TY_ = 0: the default tile height of the spreading pass at this M
template <int M, int TY_ = 0>
struct SpreadShape {
    static constexpr int TY = TY_ ? TY_ : cmin<2048 / M, M>();
    // padded FFT line (float2): lines 16 / TY float2 apart in the banks, so
    // that the column passes' 16-lane groups (TY lines x 16 / TY points) hit
    // distinct banks
    static constexpr int SC = M + (TY < 16 ? 16 / TY : 1);
    static constexpr int NPTS = TY * M;
    // fixed-point sums: a plane of int64 real parts and one of imaginary parts,
    // lines padded by 8 words so that consecutive lines of a window use the
    // two different halves of the LDS banks; the FFT input overlays them
    static constexpr int LS = M + 8;
    // key starts of a rotation: KEYS + 1 ints, room for the finest y-groups
    static constexpr int KEYS = bin_keys_max(M);
    // the sums (and FFT input) and the twiddle table; the staged knots follow
    static constexpr size_t FIXED = 16 * (size_t)TY * LS + 8 * (size_t)M;
    static_assert(8 * (size_t)TY * SC <= 16 * (size_t)TY * LS, "FFT input must fit over the sums");
};
constexpr int kMaxRanges = 24;  // two key ranges per z-cell of a window of <= 12 cells
constexpr int kSpreadThreads = 512;
// Widest window spread from staged window origins (see spread_staged_w8);
// tiles that span every row of the plane (TY = M) keep the knot's cell, since
// their rows wrap inside the tile.
constexpr int kWinMax = 8;
template <int M, int TYP>
__device__ __forceinline__ bool use_win(int w) {
    return SpreadShape<M, TYP>::TY < M && w <= kWinMax;
}

// z row z0 is live iff some knot's z-cell lies in z0-w/2 .. z0+w/2-1 on the
// periodic axis; bs are the rotation's key starts (with y-groups of 2^ygs
// cells, z-cell c owns the keys c*NYB .. c*NYB+NYB-1, NYB = M >> ygs).
template <int M>
__device__ __forceinline__ bool zrow_live(const int* __restrict__ bs, int64_t nk, int w, int z0, int ygs) {
    const int NYB = M >> ygs;
    if (nk == 0) return false;
    const int zlo = z0 - w / 2, zhi = z0 + w / 2 - 1;
    if (zlo < 0) return bs[M * NYB] - bs[(zlo + M) * NYB] + bs[(zhi + 1) * NYB] - bs[0] > 0;
    if (zhi >= M) return bs[M * NYB] - bs[zlo * NYB] + bs[(zhi - M + 1) * NYB] - bs[0] > 0;
    return bs[(zhi + 1) * NYB] - bs[zlo * NYB] > 0;
}

// Staged knot: packed cell, sorted position, window weights along x and y, the
// z weight of the tile's row, and (per component pair) the two component
// weights times the z weight and the fixed-point scale.
struct SpreadStage {
    float2* wq;  // [cap]
    int* cell;   // [cap]
    int* pos;    // [cap]
    float* wz;   // [cap]
    float* wx;   // [cap][w]
    float* wy;   // [cap][w]
};

// Key range j (0 .. 2w-1) of a tile's candidate knots, [start, start + len):
// z-cell j/2 of the z row's window and, of the y-groups that hold y-cells whose
// windows reach rows y0 .. y0+TY-1, the piece j%2 (the groups wrap around the
// periodic axis at most once).
template <int M, int TYP>
__device__ __forceinline__ void tile_range(const int* __restrict__ bs, int w, int y0, int z0, int j, int ygs,
                                           int& start, int& len) {
    using SS = SpreadShape<M, TYP>;
    constexpr int TY = SS::TY;
    const int NYB = M >> ygs;  // groups of 2^ygs y-cells; every numerator below is >= 0
    const int zc = (z0 - w / 2 + (j >> 1) + M) & (M - 1);
    const int ylo = y0 - w / 2, yhi = y0 + TY + w / 2 - 2;
    int ga[2] = {0, 0}, gb[2] = {NYB - 1, -1};  // inclusive group ranges; gb < ga is empty
    if (TY + w - 1 < M) {
        if (ylo < 0) {
            ga[0] = (ylo + M) >> ygs; gb[1] = yhi >> ygs;
        } else if (yhi >= M) {
            ga[0] = ylo >> ygs; gb[1] = (yhi - M) >> ygs;
        } else {
            ga[0] = ylo >> ygs; gb[0] = yhi >> ygs;
        }
        if (gb[1] >= ga[0]) {  // the two pieces meet: every group
            ga[0] = 0; gb[0] = NYB - 1; gb[1] = -1;
        }
    }
    const int part = j & 1;
    start = 0;
    len = 0;
    if (gb[part] >= ga[part]) {
        start = bs[zc * NYB + ga[part]];
        len = bs[zc * NYB + gb[part] + 1] - start;
    }
}

// All key ranges of a tile, by wave 0: rstart[r], and the prefix sums
// rpre[0..2w] of their lengths.
template <int M, int TYP>
__device__ void tile_ranges(const int* __restrict__ bs, int w, int y0, int z0, int ygs, int* rstart, int* rpre) {
    const int lane = threadIdx.x & 63;
    if (threadIdx.x >= 64) return;
    int start = 0, len = 0;
    if (lane < 2 * w) tile_range<M, TYP>(bs, w, y0, z0, lane, ygs, start, len);
    int incl = len;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        const int v = __shfl_up(incl, d, 64);
        if (lane >= d) incl += v;
    }
    if (lane < 2 * w) {
        rstart[lane] = start;
        rpre[lane + 1] = incl;
    }
    if (lane == 0) rpre[0] = 0;
}

// ---------------------------------------------------------------------------
// Live-tile plan of a spreading pass.  Every tile's candidate count comes from
// the key starts; tiles without candidates are marked dead and the others are
// appended to one of kPlanBuckets lists by the size of their candidate set
// (bucket b holds counts in [2^(b+3), 2^(b+4)), the first and the last
// open-ended), so that the spreading workgroups take the largest tiles first.
// plan[0 .. kPlanBuckets) are the bucket sizes and plan[kPlanBuckets] the
// spreading pass's work counter; the bin scan zeroes them.  A list entry is
// rotation * tiles + tile, tile = z row * (M / TY) + y tile.
// ---------------------------------------------------------------------------
constexpr int kPlanBuckets = plan_buckets();

template <int M, int TYP>
__device__ __forceinline__ void tile_plan(int tile, int s, const int* __restrict__ bin_start, int w, int ygs,
                                          unsigned char* __restrict__ tile_live, int* __restrict__ plan,
                                          int* __restrict__ list, int list_cap) {
    using SS = SpreadShape<M, TYP>;
    constexpr int TY = SS::TY, NTY = M / TY, TILES = M * NTY;
    const int lane = threadIdx.x & 63;
    int bucket = -1;
    if (tile < TILES) {
        const int* bs = bin_start + (size_t)s * (SS::KEYS + 1);
        const int z0 = tile / NTY, y0 = (tile % NTY) * TY;
        int ncand = 0;
        for (int j = 0; j < 2 * w; ++j) {
            int st0, len;
            tile_range<M, TYP>(bs, w, y0, z0, j, ygs, st0, len);
            ncand += len;
        }
        if (ncand == 0) tile_live[(size_t)s * TILES + tile] = 0;
        else bucket = min(max(31 - __clz(ncand) - 3, 0), kPlanBuckets - 1);
    }
    // one atomic per (wave, bucket)
    unsigned long long todo = __ballot(bucket >= 0);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int b = __shfl(bucket, leader, 64);
        const unsigned long long same = __ballot(bucket == b);
        int base = 0;
        if (lane == leader) base = atomicAdd(&plan[b], __popcll(same));
        base = __shfl(base, leader, 64);
        if (bucket == b) list[(size_t)b * list_cap + base + __popcll(same & ((1ull << lane) - 1ull))] = s * TILES + tile;
        todo &= ~same;
    }
}

// The scatter of the sorted records (workgroups x < nscatter) and the live-tile
// plan (the others) of one spreading pass, both reading the key starts.
template <int M, int TYP>
__global__ __launch_bounds__(256) void k_scatter_plan(const int4* __restrict__ rec,
                                                      const float* __restrict__ wts, const int* __restrict__ rank,
                                                      const int* __restrict__ bin_start, int64_t nk, int yshift,
                                                      int nyb, int w, float beta, float inv_i0beta, int q,
                                                      int* __restrict__ scell,
                                                      float* __restrict__ skbw, float* __restrict__ swts,
                                                      int nscatter, unsigned char* __restrict__ tile_live,
                                                      int* __restrict__ plan, int* __restrict__ list, int list_cap) {
    const int s = blockIdx.y;
    if ((int)blockIdx.x < nscatter) {
        const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
        if (j < nk)
            bin_scatter(j, s, rec, wts, rank, bin_start, nk, SpreadShape<M, TYP>::KEYS, yshift, nyb, w, beta, inv_i0beta,
                        q, scell, skbw, swts);
        return;
    }
    tile_plan<M, TYP>(((int)blockIdx.x - nscatter) * 256 + threadIdx.x, s, bin_start, w, yshift, tile_live, plan, list,
                 list_cap);
}

// Stage one block of a tile's candidates, [cbeg, cbeg + cnt) of the
// concatenated key ranges (cnt <= cap <= the workgroup size): those whose
// window reaches the tile's rows are compacted in order (wave ballots + a
// block scan) into the staging area with their cell (or window origin), sorted
// position, window weights along x and y, the z weight of the tile's row, and
// the component weights of the pair starting at component cp times that z
// weight and the fixed-point scale.  Returns how many were kept.  Every load
// of a candidate is issued at once, before it is known to be kept: the z
// weight's index follows from the key range the candidate came from (range j
// holds z-cell z0 - w/2 + j/2, whose window weight at row z0 is entry
// w - 1 - j/2), so a block costs one round trip to memory.  A block never
// holds more than the staging area, so a tile of many candidates is spread
// block by block and no candidate is ever scanned twice for one component
// pair.  Entered and left by the whole workgroup.
template <int M, int TYP, int W>
__device__ int stage_block(const int* __restrict__ sc_, const float* __restrict__ kb_,
                           const float* __restrict__ wq_, int q, int cp, float fix_scale, int y0,
                           const int* rstart, const int* rpre, int cbeg, int cnt, SpreadStage st,
                           int* wave_tot) {
    constexpr int TY = SpreadShape<M, TYP>::TY, LO = W / 2 - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int p = 0, packed = 0;
    bool keep = false;
    float2 kx[W / 2], ky[W / 2], wq2 = make_float2(0.f, 0.f);
    float wz = 0.f;
    if ((int)threadIdx.x < cnt) {
        const int ci = cbeg + (int)threadIdx.x;
        // the range holding ci, rpre[r0] <= ci < rpre[r0 + 1]: the count of the
        // (nondecreasing) prefix sums past the first that are <= ci, from
        // independent reads rather than a chain of dependent ones
        int r0 = 0;
#pragma unroll
        for (int r = 1; r < 2 * W; ++r) r0 += rpre[r] <= ci ? 1 : 0;
        p = rstart[r0] + (ci - rpre[r0]);
        packed = sc_[p];
        const float2* kw = reinterpret_cast<const float2*>(kb_ + (int64_t)p * 3 * W);
#pragma unroll
        for (int d = 0; d < W / 2; ++d) {
            kx[d] = kw[d];
            ky[d] = kw[W / 2 + d];
        }
        wz = kb_[(int64_t)p * 3 * W + 2 * W + (W - 1 - (r0 >> 1))];
        const float* wp = wq_ + (int64_t)p * q + cp;
        wq2 = make_float2(wp[0], cp + 1 < q ? wp[1] : 0.0f);
        const int cy = (packed >> 10) & 1023;
        const int ry = (cy - LO - y0 + 2 * M) & (M - 1);
        keep = ry < TY || ry > M - W;
    }
    const unsigned long long mask = __ballot(keep);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wave] = __popcll(mask);
    __syncthreads();
    int off = 0, total = 0;
#pragma unroll
    for (int v = 0; v < kSpreadThreads / 64; ++v) {
        off += v < wave ? wave_tot[v] : 0;
        total += wave_tot[v];
    }
    if (keep) {
        const int rk = off + before;
        if (use_win<M, TYP>(W)) {
            // window origin relative to the tile: first row by (signed), first
            // column bx; point (dy, dx) adds at row by + dy, column bx + dx
            const int cy = (packed >> 10) & 1023, cx = packed & 1023;
            const int ry = (cy - LO - y0 + 2 * M) & (M - 1);
            const int by = ry < TY ? ry : ry - M;
            const int bx = (cx - LO + M) & (M - 1);
            st.cell[rk] = ((by * SpreadShape<M, TYP>::LS + bx) & 0xffff) | (by << 16);
        } else {
            st.cell[rk] = packed;
        }
        st.pos[rk] = p;
        float2* dx = reinterpret_cast<float2*>(st.wx + rk * W);
        float2* dy = reinterpret_cast<float2*>(st.wy + rk * W);
#pragma unroll
        for (int d = 0; d < W / 2; ++d) {
            dx[d] = kx[d];
            dy[d] = ky[d];
        }
        st.wz[rk] = wz;
        const float f = wz * fix_scale;
        st.wq[rk] = make_float2(wq2.x * f, wq2.y * f);
    }
    __syncthreads();
    return total;
}

// Exact int64 -> double split (hi * 2^32 + lo), then one rounding to float.
__device__ __forceinline__ float fixed_to_float(unsigned long long u, float inv) {
    const long long x = (long long)u;
    const double d = fma((double)(int)(x >> 32), 4294967296.0, (double)(unsigned)(x & 0xffffffffull));
    return (float)(d * (double)inv);
}

// The staged knots of one block, spread for one component pair into the two
// planes of fixed-point sums.  Each wave takes U staged knots at a time (every
// NW-th), a lane per window point, w^2 points per knot: the LDS reads of all U
// are issued together, then the atomic adds of the lanes that land in the
// tile.  Used where w^2 fills whole waves (w = 8) or nearly (w = 10).  The sums
// are exact integers, so the order of the adds does not matter.
template <int M, int TYP>
__device__ __forceinline__ void spread_staged_rows(const SpreadStage& st, int nst, int w, int y0,
                                                   unsigned long long* __restrict__ acc) {
    using SS = SpreadShape<M, TYP>;
    constexpr int TY = SS::TY, LS = SS::LS, NW = kSpreadThreads / 64, U = 4;
    const int lo = w / 2 - 1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int dmul = (65536 + w - 1) / w;  // t / w for t < w*w by a multiply
    for (int i0 = wave; i0 < nst; i0 += U * NW) {
        for (int t0 = 0; t0 < w * w; t0 += 64) {
            const int t = t0 + lane;
            const int ddy = min((t * dmul) >> 16, w - 1), ddx = t - ((t * dmul) >> 16) * w;
            int packed[U];
            float wyx[U];
            float2 c2[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = min(i0 + u * NW, nst - 1);
                packed[u] = st.cell[i];
                wyx[u] = st.wy[i * w + ddy] * st.wx[i * w + ddx];
                c2[u] = st.wq[i];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int cx = packed[u] & 1023, cy = (packed[u] >> 10) & 1023;
                const int l = (cy - lo - y0 + ddy + 2 * M) & (M - 1);
                if (i0 + u * NW < nst && t < w * w && l < TY) {
                    const int off = l * LS + ((cx - lo + ddx + M) & (M - 1));
                    // |addend| <= 2^30: a 32-bit conversion, sign-extended
                    atomicAdd(acc + off, (unsigned long long)(long long)__float2int_rn(c2[u].x * wyx[u]));
                    atomicAdd(acc + TY * LS + off,
                              (unsigned long long)(long long)__float2int_rn(c2[u].y * wyx[u]));
                }
            }
        }
    }
}

// Windows of w <= kWinMax on tiles of fewer rows than the plane use a staged
// window origin instead of the knot's cell: its first row by relative to the tile (-(w-1) .. TY-1) and its first
// column bx (0 .. M-1), packed as (by * LS + bx) in the low 16 bits (two's
// complement) and by in the high 16.  Window point (dy, dx) then adds at LDS
// word (by * LS + bx) + (dy * LS + dx), with no wrap: a line's columns
// M .. M+w-2 (inside its padding, LS - M = 8 >= w - 1) collect the points past
// the periodic edge and are folded back onto columns 0 .. w-2 before the
// transform.
__device__ __forceinline__ int win_row(int word) { return word >> 16; }
__device__ __forceinline__ int win_off(int word) { return (int)(short)(word & 0xffff); }

// w = 8: a knot's 64 window points fill a wave instruction, a lane per point
// (row lane / 8, column lane % 8).  Each wave takes U staged knots at a time
// (every NW-th); their LDS reads are issued together, then the atomic adds of
// the lanes whose row lies in the tile.
template <int M, int TYP>
__device__ __forceinline__ void spread_staged_w8(const SpreadStage& st, int nst,
                                                 unsigned long long* __restrict__ acc) {
    using SS = SpreadShape<M, TYP>;
    constexpr int TY = SS::TY, LS = SS::LS, NW = kSpreadThreads / 64, U = 4, W = 8;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ddy = lane >> 3, ddx = lane & 7, loff = ddy * LS + ddx;
    for (int i0 = wave; i0 < nst; i0 += U * NW) {
        int word[U];
        float wyx[U];
        float2 c2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = min(i0 + u * NW, nst - 1);
            word[u] = st.cell[i];
            wyx[u] = st.wy[i * W + ddy] * st.wx[i * W + ddx];
            c2[u] = st.wq[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i0 + u * NW < nst && (unsigned)(win_row(word[u]) + ddy) < (unsigned)TY) {
                const int off = win_off(word[u]) + loff;
                // |addend| <= 2^30: a 32-bit conversion, sign-extended
                atomicAdd(acc + off, (unsigned long long)(long long)__float2int_rn(c2[u].x * wyx[u]));
                atomicAdd(acc + TY * LS + off, (unsigned long long)(long long)__float2int_rn(c2[u].y * wyx[u]));
            }
        }
    }
}

// w = 6: a wave instruction takes two window rows of five knots (2 rows x 6
// columns each, 60 of 64 lanes): lane l serves knot l / 12 of a group, row
// (l % 12) / 6 (then + 2 and + 4 in the next two instructions), column l % 6.
// The two rows of one knot in an instruction are consecutive lines, which lie
// in different halves of the LDS banks.  Each wave takes U groups at a time
// (every NW-th).
template <int M, int TYP>
__device__ __forceinline__ void spread_staged_w6(const SpreadStage& st, int nst,
                                                 unsigned long long* __restrict__ acc) {
    using SS = SpreadShape<M, TYP>;
    constexpr int TY = SS::TY, LS = SS::LS, NW = kSpreadThreads / 64, U = 1, W = 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = lane / 12, r = lane - slot * 12, ddy = r / W, ddx = r - ddy * W;
    const int loff = ddy * LS + ddx;
    const int ngrp = (nst + 4) / 5;
    for (int g0 = wave; g0 < ngrp; g0 += U * NW) {
        int word[U];
        bool ok[U];
        float wy[U][3], wx[U];
        float2 c2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = (g0 + u * NW) * 5 + slot;
            ok[u] = slot < 5 && i < nst;
            const int ic = min(i, nst - 1);  // a valid index for the reads
            word[u] = st.cell[ic];
#pragma unroll
            for (int p = 0; p < 3; ++p) wy[u][p] = st.wy[ic * W + 2 * p + ddy];
            wx[u] = st.wx[ic * W + ddx];
            c2[u] = st.wq[ic];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            const int row = win_row(word[u]) + ddy, off = win_off(word[u]) + loff;
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                if ((unsigned)(row + 2 * p) < (unsigned)TY) {
                    const float f = wy[u][p] * wx[u];
                    atomicAdd(acc + off + 2 * p * LS, (unsigned long long)(long long)__float2int_rn(c2[u].x * f));
                    atomicAdd(acc + TY * LS + off + 2 * p * LS,
                              (unsigned long long)(long long)__float2int_rn(c2[u].y * f));
                }
            }
        }
    }
}

// Zero both planes of fixed-point sums (2 * PAIRS 64-bit words), 16 bytes a store.
template <int PAIRS, int NT>
__device__ __forceinline__ void clear_sums(unsigned long long* acc) {
    ulonglong2* p = reinterpret_cast<ulonglong2*>(acc);
    for (int t = threadIdx.x; t < PAIRS; t += NT) p[t] = make_ulonglong2(0ull, 0ull);
}

// One spreading tile (z row z0, y rows y0 .. y0+TY-1 of rotation s), for the
// components c0 .. c1-1 (c0 even).  Entered by the whole workgroup; the LDS
// regions are laid out by the caller.
template <int M, int TYP>
__device__ bool spread_tile(int s, int z0, int y0, int yt, int c0, int c1, const int* __restrict__ bin_start,
                            unsigned char* __restrict__ tile_live, const int* __restrict__ scell,
                            const float* __restrict__ skbw, const float* __restrict__ swts, int64_t nk, int q, int w,
                            int cap, float fix_scale, float fix_inv, float2* __restrict__ out, float2* lds,
                            int* wave_tot, int* rstart, int* rpre, int ygs) {
    constexpr int H = M / 4;  // half of the n = M/2 kept modes along x
    using SS = SpreadShape<M, TYP>;
    constexpr int TY = SS::TY, SC = SS::SC, NPTS = SS::NPTS, LS = SS::LS;
    constexpr int NT = kSpreadThreads;
    static_assert(NPTS % NT == 0, "tile must split evenly over the workgroup");
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(lds);  // [2][TY][LS]
    float2* a = lds;                                                       // [TY][SC] over the sums
    float2* twl = lds + 2 * TY * LS;                                       // after both planes
    SpreadStage st;
    st.wq = twl + M;
    st.cell = reinterpret_cast<int*>(st.wq + cap);
    st.pos = st.cell + cap;
    st.wz = reinterpret_cast<float*>(st.pos + cap);
    st.wx = st.wz + cap;
    st.wy = st.wx + cap * w;
    const int nr = 2 * w;
    const int* sc_ = scell + (int64_t)s * nk;
    const float* kb_ = skbw + (int64_t)s * nk * 3 * w;
    const float* wq_ = swts + (int64_t)s * nk * q;
    if (c0 >= c1) return false;  // no component to spread (never staged: weights would be read past q)
    tile_ranges<M, TYP>(bin_start + (size_t)s * (SS::KEYS + 1), w, y0, z0, ygs, rstart, rpre);
    __syncthreads();
    const int ncand = rpre[nr];
    // candidates are spread in blocks of `cap` (one staging each): a tile of one
    // block is staged once for all its component pairs, a tile of several is
    // staged block by block for each pair
    const int nblk = (ncand + cap - 1) / cap;
    auto stage = [&](int b, int cp) {
        const int c0b = b * cap, cnt = min(cap, ncand - b * cap);
        switch (w) {  // the width as a constant: the loaded weights stay in registers
        case 6: return stage_block<M, TYP, 6>(sc_, kb_, wq_, q, cp, fix_scale, y0, rstart, rpre, c0b, cnt, st, wave_tot);
        case 8: return stage_block<M, TYP, 8>(sc_, kb_, wq_, q, cp, fix_scale, y0, rstart, rpre, c0b, cnt, st, wave_tot);
        case 10: return stage_block<M, TYP, 10>(sc_, kb_, wq_, q, cp, fix_scale, y0, rstart, rpre, c0b, cnt, st,
                                           wave_tot);
        default: return stage_block<M, TYP, 12>(sc_, kb_, wq_, q, cp, fix_scale, y0, rstart, rpre, c0b, cnt, st,
                                           wave_tot);
        }
    };
    int kept = nblk == 1 ? stage(0, c0) : 0;  // the single block, staged with the first pair's weights
    if (ncand == 0 || (nblk == 1 && kept == 0)) {
        if (threadIdx.x == 0) tile_live[((size_t)s * M + z0) * (M / TY) + yt] = 0;
        return false;  // no knot reaches the tile: its spectrum is zero and is not written
    }
    int kept_all = 0;  // knots of the tile (counted while spreading the first pair)
    clear_sums<TY * LS, NT>(acc);
    for (int cp = c0; cp < c1; cp += 2) {
        // with one block, the next pair's weights are read (a thread per staged
        // knot) while this pair is spread
        const bool prefetch = nblk == 1 && cp + 2 < c1 && (int)threadIdx.x < kept;
        float2 nxt = make_float2(0.f, 0.f);
        static_assert(kSpreadThreads >= 512, "one staged knot per thread");
        for (int b = 0; b < nblk; ++b) {
            if (nblk > 1) kept = stage(b, cp);  // ends with a barrier
            else __syncthreads();               // the staged weights (first pair) or the prefetched ones
            if (cp == c0) kept_all += kept;
            if (prefetch) {
                const float* wp = wq_ + (int64_t)st.pos[threadIdx.x] * q + cp + 2;
                const float f = st.wz[threadIdx.x] * fix_scale;
                nxt = make_float2(wp[0] * f, cp + 3 < q ? wp[1] * f : 0.0f);
            }
            if (use_win<M, TYP>(w) && w == 6) spread_staged_w6<M, TYP>(st, kept, acc);
            else if (use_win<M, TYP>(w) && w == 8) spread_staged_w8<M, TYP>(st, kept, acc);
            else spread_staged_rows<M, TYP>(st, kept, w, y0, acc);
            __syncthreads();
        }
        if (cp == c0) {
            // a tile whose candidates all miss its rows: dead, nothing written
            if (threadIdx.x == 0) tile_live[((size_t)s * M + z0) * (M / TY) + yt] = kept_all > 0;
            if (kept_all == 0) return false;
        }
        if (prefetch) st.wq[threadIdx.x] = nxt;  // read from the next pair on, after the barriers below
        // sums -> FFT input over the same memory, fused with the first radix-8
        // pass of the x transform: each thread converts the eight points of its
        // first butterfly and transforms them in registers.  With window
        // origins, the points past the periodic edge (columns M .. M+w-2) are
        // added back onto columns 0 .. w-2 here, as integers.
        {
            constexpr int NB0 = M / 8, WORK0 = TY * NB0;
            static_assert(WORK0 <= NT, "one first-pass butterfly per thread");
            int c = threadIdx.x % TY, jb = threadIdx.x / TY;
            if constexpr (NB0 >= 8 && TY % 2 == 0) {
                // a 16-lane group takes two rows and eight consecutive
                // butterflies, so that its reads of the sums fall in distinct banks
                constexpr int NRP = TY / 2;
                const int l = threadIdx.x & 15, g = threadIdx.x >> 4;
                c = 2 * (g % NRP) + (l >> 3);
                jb = 8 * (g / NRP) + (l & 7);
            }
            const bool fold = use_win<M, TYP>(w);
            float2 v0[8];
            if ((int)threadIdx.x < WORK0) {
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int e = c * LS + jb + r * NB0;
                    unsigned long long re = acc[e], im = acc[TY * LS + e];
                    if (fold && jb + r * NB0 < w - 1) {
                        re += acc[c * LS + M + jb + r * NB0];
                        im += acc[TY * LS + c * LS + M + jb + r * NB0];
                    }
                    v0[r] = make_float2(fixed_to_float(re, fix_inv), fixed_to_float(im, fix_inv));
                }
                dft8<-1>(v0);
            }
            __syncthreads();
            if ((int)threadIdx.x < WORK0) {
#pragma unroll
                for (int r = 0; r < 8; ++r) a[c * SC + jb * 8 + r] = v0[r];
            }
            __syncthreads();
        }
        fft_passes<M, 8, -1, TY, 1, SC, NT, true>(a, twl);  // only the kept band is read below
        // both half spectra of a mode from one read of its two entries
        constexpr int PER = TY * H;
        const bool second = cp + 1 < q;
        for (int t = threadIdx.x; t < PER; t += NT) {
            const int l = t / H, mm = t % H;
            const float2 z1 = a[l * SC + mm];
            const float2 z2 = a[l * SC + ((M - mm) & (M - 1))];
            float2* o = out + ((((size_t)s * q + cp) * M + z0) * M + y0 + l) * H + mm;
            o[0] = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y));
            if (second) o[(size_t)M * M * H] = make_float2(0.5f * (z1.y + z2.y), 0.5f * (z2.x - z1.x));
        }
        if (cp + 2 < c1) {
            __syncthreads();
            clear_sums<TY * LS, NT>(acc);
        }
    }
    return true;
}

// Persistent spreading pass: each workgroup takes work items of the plan's
// lists (largest candidate sets first) from a shared counter until none are
// left.  An item is a tile, or, when the pass has fewer live tiles than twice
// the workgroups, a tile of the buckets from kSplitBucket up is cut into one
// item per component pair: the heaviest tiles then no longer set the pass's
// length.  Each pair's output is written by one item only, with exact sums, so
// the result does not depend on the cut.
constexpr int kSplitBucket = 5;  // candidate sets of 256 knots or more
constexpr int kSplitParts = 5;   // items per cut tile (at most the component pairs)

template <int M, int TYP>
__global__ __launch_bounds__(kSpreadThreads, 4) void k_spread_fftx(const int* __restrict__ bin_start,
                                                                unsigned char* __restrict__ tile_live,
                                                                int* __restrict__ plan, const int* __restrict__ list,
                                                                int list_cap, const int* __restrict__ scell,
                                                                const float* __restrict__ skbw,
                                                                const float* __restrict__ swts, int64_t nk, int q,
                                                                int w, int cap, float fix_scale, float fix_inv,
                                                                float2* __restrict__ out,
                                                                const float2* __restrict__ twm,
                                                                unsigned long long* __restrict__ work,
                                                                unsigned long long rec_bytes, int ygs) {
    using SS = SpreadShape<M, TYP>;
    constexpr int NTY = M / SS::TY, TILES = M * NTY;
    unsigned long long wrote = 0;  // bytes of kept x modes this workgroup wrote
    extern __shared__ float2 lds[];
    __shared__ int wave_tot[kSpreadThreads / 64];
    __shared__ int rstart[kMaxRanges], rpre[kMaxRanges + 1];
    __shared__ int first[kPlanBuckets], size[kPlanBuckets], parts[kPlanBuckets], cur, total;
    load_table<M, kSpreadThreads>(lds + 2 * SS::TY * SS::LS, twm);
    if (threadIdx.x == 0) {
        int tiles = 0;
        for (int b = 0; b < kPlanBuckets; ++b) tiles += plan[b];
        const bool cut = tiles < 2 * (int)gridDim.x;
        int run = 0;
        for (int b = kPlanBuckets - 1; b >= 0; --b) {
            first[b] = run;
            size[b] = plan[b];
            // every part gets at least one component pair: with ppp pairs per
            // part, only ceil(pairs / ppp) parts are needed (6 pairs in at most
            // 5 parts are 3 parts of 2)
            const int pairs = (q + 1) / 2, ppp = (pairs + min(kSplitParts, pairs) - 1) / min(kSplitParts, pairs);
            parts[b] = cut && b >= kSplitBucket ? (pairs + ppp - 1) / ppp : 1;
            run += size[b] * parts[b];
        }
        total = run;
    }
    for (;;) {
        if (threadIdx.x == 0) cur = atomicAdd(&plan[kPlanBuckets], 1);
        __syncthreads();
        const int k = cur;
        if (k >= total) break;
        int b = kPlanBuckets - 1;
        while (k >= first[b] + size[b] * parts[b]) --b;
        const int e = (k - first[b]) / parts[b], part = (k - first[b]) % parts[b];
        const int id = list[(size_t)b * list_cap + e];
        const int s = id / TILES, tile = id % TILES;
        const int ppp = ((q + 1) / 2 + parts[b] - 1) / parts[b];  // component pairs per part
        const int c0 = 2 * part * ppp, c1 = min(c0 + 2 * ppp, q);  // c0 < q: no part is empty
        if (spread_tile<M, TYP>(s, tile / NTY, (tile % NTY) * SS::TY, tile % NTY, c0, c1, bin_start, tile_live, scell,
                           skbw, swts, nk, q, w, cap, fix_scale, fix_inv, out, lds, wave_tot, rstart, rpre, ygs))
            wrote += (unsigned long long)SS::TY * (M / 4) * sizeof(float2) * (c1 - c0);
    }
    // work record, summed over launches until the host reads it: bytes of kept
    // x modes written, sorted knot records read, launches
    if (threadIdx.x == 0) {
        if (wrote) atomicAdd(work, wrote);
        if (blockIdx.x == 0) {
            atomicAdd(work + 1, rec_bytes);
            atomicAdd(work + 2, 1ull);
        }
    }
}

// Index of kept output mode o (FFT order of an n-point axis) in an m-point FFT;
// -1 for the Nyquist slot.
template <int N, int M>
__device__ __forceinline__ int kept_source(int o) {
    if (o == N / 2) return -1;
    const int mo = o < N / 2 ? o : o - N;
    return (mo + M) & (M - 1);
}

// The widths of one column pass: the default D and, where they stay within
// [LO, HI], D / 2 and 2 D (the kernels are instantiated for each).
template <int D, int LO, int HI>
struct Cols {
    static constexpr int DEF = D, DN = D / 2 >= LO ? D / 2 : D, UP = 2 * D <= HI ? 2 * D : D;
    static int list(int out[3]) {
        int k = 0;
        out[k++] = D;
        if (DN != D) out[k++] = DN;
        if (UP != D) out[k++] = UP;
        return k;
    }
};

template <int M>
struct ColShape {
    static constexpr int N = M / 2, H = N / 2;
    // column batches: a forward y workgroup of 8 columns at m = 256 (16 at 128)
    // keeps more workgroups per CU in flight than 16 (32) and was measured faster,
    // as were 16-column inverse y and 16-line-pair inverse x workgroups at
    // n = 128; the z passes keep 8
    static constexpr int COLS = cmin<H, 2048 / M>();          // forward y pass
    static constexpr int ZCOLS = cmin<H, 2048 / M>();         // z passes
    static constexpr int YZB = 1;                              // z rows per y-pass workgroup
    static constexpr int ICOLS = cmin<H, 2048 / N>();         // inverse y pass
    static constexpr int XCOLS = cmin<N * N / 2, 2048 / N>(); // inverse x pass (line pairs)
    // the widths the autotuner may choose from; the inverse x pass needs whole
    // output loops, 2 XCOLS N a multiple of the workgroup size
    using Y = Cols<COLS, 1, H>;
    using Z = Cols<ZCOLS, 1, H>;
    using IY = Cols<ICOLS, 1, H>;
    using IX = Cols<XCOLS, (128 / N > 1 ? 128 / N : 1), N * N / 2>;
};

// fft_cols (columns interleaved) with its first, radix-8 pass taken on values
// the caller already holds in registers: v[u][r] is element (row j + r LEN/8,
// column c) of the thread's u-th butterfly, t = u NT + threadIdx.x, j = t / COLS,
// c = t % COLS -- the elements that pass reads -- so the input never goes
// through LDS.  The same butterflies in the same order: the result equals
// fft_cols bit for bit.  `a` must not be read by any thread on entry.
template <int LEN, int COLS, int NT = kThreads>
struct RegPass {
    static_assert(LEN >= 8, "radix-8 first pass");
    static constexpr int NB = LEN / 8, WORK = NB * COLS, NBF = (WORK + NT - 1) / NT;
};

// Raw buffer view of one array (float2 or float): the buffer unit checks every
// offset against the array's size, and a load at or past the end returns zero
// without touching memory.  A column read that skips dead rows then needs no
// branch (offset kPastEnd), and the compiler can count the loads in flight
// exactly, so they stay in flight across the transform that follows.
constexpr uint32_t kPastEnd = 0x80000000u;
struct ZeroPastEnd {
    __amdgpu_buffer_rsrc_t r;
    // dword 3 of the resource: 32-bit data format, no swizzle, no thread id
    __device__ ZeroPastEnd(const float2* base, size_t count)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(base), 0, (int)(count * sizeof(float2)), 0x00020000)) {}
    __device__ ZeroPastEnd(const float* base, size_t count)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, (int)(count * sizeof(float)), 0x00020000)) {}
    __device__ float2 load(uint32_t byte_off) const {
        const auto d = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
        return make_float2(__uint_as_float(d[0]), __uint_as_float(d[1]));
    }
    __device__ float load1(uint32_t byte_off) const {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
    }
};

template <int LEN, int SIGN, int COLS, bool HALF, int NBF, int NT = kThreads>
__device__ __forceinline__ void fft_cols_regs_impl(float2 (&v)[NBF][8], float2* a, const float2* tw) {
    using P = RegPass<LEN, COLS, NT>;
    static_assert(NBF == P::NBF, "one register row per first-pass butterfly");
#pragma unroll
    for (int u = 0; u < P::NBF; ++u) {
        const int t = u * NT + (int)threadIdx.x;
        if (P::WORK % NT == 0 || t < P::WORK) {
            const int c = t % COLS, j = t / COLS;
            dft8<SIGN>(v[u]);
#pragma unroll
            for (int r = 0; r < 8; ++r) a[(j * 8 + r) * COLS + c] = v[u][r];
        }
    }
    __syncthreads();
    fft_passes<LEN, 8, SIGN, COLS, COLS, 1, NT, HALF>(a, tw);
}
template <int LEN, int SIGN, int COLS, int NBF>
__device__ __forceinline__ void fft_cols_regs(float2 (&v)[NBF][8], float2* a, const float2* tw) {
    fft_cols_regs_impl<LEN, SIGN, COLS, false>(v, a, tw);
}
// The same, with only the band of outputs the forward passes keep (index
// < LEN/4 or >= 3 LEN/4) written; bit for bit the same values there.
template <int LEN, int SIGN, int COLS, int NBF>
__device__ __forceinline__ void fft_cols_regs_band(float2 (&v)[NBF][8], float2* a, const float2* tw) {
    fft_cols_regs_impl<LEN, SIGN, COLS, true>(v, a, tw);
}

// a2: y pass over [slab][z][y][mx] -> [slab][z][my][mx], M points pruned to N,
// slab = rotation * q + component.  A workgroup takes YZB z rows of one
// rotation and column block, every component of them; dead z rows are skipped
// (their output is never read) and rows of dead y tiles are zero.
template <int M, int COLS, int TYP>
__global__ __launch_bounds__(kThreads) void k_fft_y(const float2* __restrict__ in, float2* __restrict__ out,
                                                    const float2* __restrict__ twm, int q, int cg,
                                                    const int* __restrict__ bin_start,
                                                    const unsigned char* __restrict__ tile_live, int64_t nk, int w,
                                                    int ygs) {
    constexpr int N = ColShape<M>::N, H = ColShape<M>::H, YZB = ColShape<M>::YZB;
    constexpr int TY = SpreadShape<M, TYP>::TY, NT = M / TY;
    using P = RegPass<M, COLS>;
    extern __shared__ float2 lds[];
    __shared__ unsigned char live[NT];
    float2* a = lds;
    float2* twl = a + M * COLS;
    // one workgroup per (column block, z row, rotation, group of cg
    // components): the group's components of the row are transformed in turn,
    // the next one's columns read into registers while the current one is
    // transformed
    const int ng = (q + cg - 1) / cg;
    const int s = blockIdx.z / ng, cbeg = (blockIdx.z % ng) * cg, cend = min(q, cbeg + cg);
    const int* bs = bin_start + (size_t)s * (SpreadShape<M, TYP>::KEYS + 1);
    const int c0 = blockIdx.x * COLS;
    load_table<M>(twl, twm);
    for (int z = blockIdx.y * YZB; z < blockIdx.y * YZB + YZB; ++z) {
        if (!zrow_live<M>(bs, nk, w, z, ygs)) continue;
        __syncthreads();  // the previous row's output has been read out of `a`
        for (int t = threadIdx.x; t < NT; t += kThreads) live[t] = tile_live[((size_t)s * M + z) * NT + t];
        __syncthreads();
        float2 nxt[P::NBF][8];
        auto fetch = [&](int c) {
            const float2* src = in + ((size_t)(s * q + c) * M + z) * M * H + c0;
#pragma unroll
            for (int u = 0; u < P::NBF; ++u) {
                const int t = u * kThreads + (int)threadIdx.x;
                if (P::WORK % kThreads == 0 || t < P::WORK) {
                    const int cc = t % COLS, j = t / COLS;
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        const int y = j + r * P::NB;
                        nxt[u][r] = live[y / TY] ? src[(size_t)y * H + cc] : make_float2(0.f, 0.f);
                    }
                }
            }
        };
        fetch(cbeg);
        for (int c = cbeg; c < cend; ++c) {
            float2 v[P::NBF][8];
#pragma unroll
            for (int u = 0; u < P::NBF; ++u)
#pragma unroll
                for (int r = 0; r < 8; ++r) v[u][r] = nxt[u][r];
            if (c + 1 < cend) fetch(c + 1);
            fft_cols_regs_band<M, -1, COLS>(v, a, twl);
            float2* dst = out + ((size_t)(s * q + c) * M + z) * N * H + c0;
            for (int t = threadIdx.x; t < N * COLS; t += kThreads) {
                const int o = t / COLS, cc = t % COLS;
                const int si = kept_source<N, M>(o);
                dst[(size_t)o * H + cc] = si < 0 ? make_float2(0.f, 0.f) : a[si * COLS + cc];
            }
            __syncthreads();  // `a` read out before the next component's transform
        }
    }
}

// Shared part of the z pass: transform each component's z-columns for one my
// row and accumulate sum_c vtab[c][|m|^2] * G_c into per-thread registers
// (thread t holds entries t + k*kThreads of the [mz][col] block).
template <int M, int COLS>
struct ZAcc {
    static constexpr int N = M / 2;
    static constexpr int PER = (N * COLS + kThreads - 1) / kThreads;
};

// zlive[z] (LDS) tells which z rows the y pass wrote; the others are zero.
template <int M, int COLS>
__device__ __forceinline__ void z_accumulate(const float2* __restrict__ in, int s, int q, int iy, int c0,
                                             const float* __restrict__ vtab, int m2n, float2* a,
                                             const float2* twl, const unsigned char* zlive,
                                             float2 (&acc)[ZAcc<M, COLS>::PER]) {
    constexpr int N = ColShape<M>::N, H = ColShape<M>::H, PER = ZAcc<M, COLS>::PER;
    using P = RegPass<M, COLS>;
    const int my = iy < N / 2 ? iy : iy - N;
#pragma unroll
    for (int k = 0; k < PER; ++k) acc[k] = make_float2(0.f, 0.f);
    // the kept outputs' ball-transform entries: index |m|^2, or -1
    int vidx[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x + k * kThreads;
        const int o = t / COLS, cc = t % COLS;
        const int mz = o < N / 2 ? o : o - N, mx = c0 + cc;
        const bool kept = t < N * COLS && kept_source<N, M>(o) >= 0;
        vidx[k] = kept ? mx * mx + my * my + mz * mz : -1;
    }
    // component c's columns (in the order of the transform's first pass) and
    // its ball-transform entries are read into registers while component c-1
    // is being transformed: two register sets in turn.  Every read is issued
    // unconditionally (dead rows, outputs out of the band and components past
    // the last one read zeros past the end of a buffer view), so the loads of
    // the next component stay in flight through the whole transform.
    float2 va[P::NBF][8], vb[P::NBF][8];
    float wa[PER], wb[PER];
    auto fetch = [&](float2 (&v)[P::NBF][8], float (&wt)[PER], int c) {
        const bool ok = c < q;
        const int cs = ok ? c : q - 1;
        const ZeroPastEnd vt(vtab + (size_t)cs * m2n, ok ? (size_t)m2n : 0);
#pragma unroll
        for (int k = 0; k < PER; ++k) wt[k] = vt.load1(vidx[k] >= 0 ? (uint32_t)vidx[k] * 4u : kPastEnd);
        const ZeroPastEnd src(in + (((size_t)s * q + cs) * M) * N * H + (size_t)iy * H + c0,
                              ok ? (size_t)M * N * H - (size_t)iy * H - c0 : 0);
#pragma unroll
        for (int u = 0; u < P::NBF; ++u) {
            const int t = u * kThreads + (int)threadIdx.x;
            if (P::WORK % kThreads == 0 || t < P::WORK) {
                const int cc = t % COLS, j = t / COLS;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int z = j + r * P::NB;
                    v[u][r] = src.load(zlive[z] ? (uint32_t)(z * N * H + cc) * 8u : kPastEnd);
                }
            }
        }
    };
    auto transform = [&](float2 (&v)[P::NBF][8], const float (&wt)[PER]) {
        fft_cols_regs_band<M, -1, COLS>(v, a, twl);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (vidx[k] >= 0) {
                const int t = threadIdx.x + k * kThreads;
                const int o = t / COLS, cc = t % COLS;
                const float2 g = a[kept_source<N, M>(o) * COLS + cc];
                acc[k].x = fmaf(wt[k], g.x, acc[k].x);
                acc[k].y = fmaf(wt[k], g.y, acc[k].y);
            }
        }
        __syncthreads();
    };
    fetch(va, wa, 0);
    for (int c = 0; c < q; c += 2) {
        fetch(vb, wb, c + 1);
        transform(va, wa);
        if (c + 1 == q) break;
        fetch(va, wa, c + 2);
        transform(vb, wb);
    }
}

// a2 (z) + a3 for the fixed shape or a single spectrum: F = D(m) * acc; with
// deconv NULL the plain sums acc (the rotated shape's z pass shared by several
// products, each finished by k_product_ifft_z).
template <int M, int COLS>
__global__ __launch_bounds__(kThreads) void k_fft_z_spectrum(const float2* __restrict__ in, int q,
                                                             const float* __restrict__ vtab, int m2n,
                                                             const double* __restrict__ deconv,
                                                             float2* __restrict__ spec, const float2* __restrict__ twm,
                                                             const int* __restrict__ bin_start, int64_t nk, int w, int ygs) {
    constexpr int N = ColShape<M>::N, H = ColShape<M>::H, PER = ZAcc<M, COLS>::PER;
    extern __shared__ float2 lds[];
    __shared__ unsigned char zlive[M];
    float2* a = lds;
    float2* twl = a + M * COLS;
    const Blk b = xcd_block();
    const int c0 = b.x * COLS, iy = b.y, s = b.z;
    float2* dst = spec + (size_t)s * N * N * H + (size_t)iy * H + c0;
    if (iy == N / 2) {
        for (int t = threadIdx.x; t < N * COLS; t += kThreads)
            dst[(size_t)(t / COLS) * N * H + t % COLS] = make_float2(0.f, 0.f);
        return;
    }
    load_table<M>(twl, twm);
    for (int t = threadIdx.x; t < M; t += kThreads) zlive[t] = zrow_live<M>(bin_start + (size_t)s * (SpreadShape<M>::KEYS + 1), nk, w, t, ygs);
    __syncthreads();
    float2 acc[PER];
    z_accumulate<M, COLS>(in, s, q, iy, c0, vtab, m2n, a, twl, zlive, acc);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x + k * kThreads;
        if (t < N * COLS) {
            const int o = t / COLS, cc = t % COLS;
            if (deconv) {
                const float d = (float)(deconv[c0 + cc] * deconv[iy] * deconv[o]);
                dst[(size_t)o * N * H + cc] = make_float2(acc[k].x * d, acc[k].y * d);
            } else {
                dst[(size_t)o * N * H + cc] = acc[k];
            }
        }
    }
}

// The product's factor prod_d D(m_d) exp(i k_d o_d) / L for output mode
// (x index cx, y index iy, z index o), from the per-axis FP64 table, as float.
__device__ __forceinline__ float2 shift_factor(const double2* __restrict__ phase, int n, int cx, int iy, int o) {
    const double2 px = phase[cx], py = phase[n + iy], pz = phase[2 * n + o];
    const double fr = px.x * py.x - px.y * py.y, fi = px.x * py.y + px.y * py.x;
    const double gr = fr * pz.x - fi * pz.y, gi = fr * pz.y + fi * pz.x;
    return make_float2((float)gr, (float)gi);
}

// a2 (z) + a3 + a4 + inverse z for the rotated shape:
//   S = F_A * conj(acc) * prod_d D(m_d) exp(i k_d o_d) / L   (factor in FP64),
// then the unnormalised inverse transform along z.
template <int M, int COLS>
__global__ __launch_bounds__(kThreads) void k_fft_z_product(const float2* __restrict__ in, int q,
                                                            const float* __restrict__ vtab, int m2n,
                                                            const double2* __restrict__ phase,
                                                            const float2* __restrict__ fa, float2* __restrict__ out,
                                                            const float2* __restrict__ twm,
                                                            const float2* __restrict__ twn,
                                                            const int* __restrict__ bin_start, int64_t nk, int w, int ygs) {
    constexpr int N = ColShape<M>::N, H = ColShape<M>::H, PER = ZAcc<M, COLS>::PER;
    extern __shared__ float2 lds[];
    __shared__ unsigned char zlive[M];
    float2* a = lds;
    float2* twl = a + M * COLS;
    float2* twnl = twl + M;
    const Blk b = xcd_block();
    const int c0 = b.x * COLS, iy = b.y, s = b.z;
    float2* dst = out + (size_t)s * N * N * H + (size_t)iy * H + c0;
    if (iy == N / 2) {
        for (int t = threadIdx.x; t < N * COLS; t += kThreads)
            dst[(size_t)(t / COLS) * N * H + t % COLS] = make_float2(0.f, 0.f);
        return;
    }
    load_table<M>(twl, twm);
    load_table<N>(twnl, twn);
    for (int t = threadIdx.x; t < M; t += kThreads) zlive[t] = zrow_live<M>(bin_start + (size_t)s * (SpreadShape<M>::KEYS + 1), nk, w, t, ygs);
    __syncthreads();
    float2 acc[PER];
    z_accumulate<M, COLS>(in, s, q, iy, c0, vtab, m2n, a, twl, zlive, acc);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int t = threadIdx.x + k * kThreads;
        if (t < N * COLS) {
            const int o = t / COLS, cc = t % COLS;
            const float2 A = fa[((size_t)o * N + iy) * H + c0 + cc];
            a[o * COLS + cc] = cmul(cmul(A, make_float2(acc[k].x, -acc[k].y)), shift_factor(phase, N, c0 + cc, iy, o));
        }
    }
    __syncthreads();
    fft_cols<N, 1, COLS, false>(a, twnl);
    for (int t = threadIdx.x; t < N * COLS; t += kThreads) dst[(size_t)(t / COLS) * N * H + t % COLS] = a[t];
}

// a4 + inverse z for one more fixed spectrum, from the rotated shape's z sums
// acc [s][mz][my][mx] (k_fft_z_spectrum without deconvolution): the same
// product and transform as k_fft_z_product, in the same order of operations.
template <int M, int COLS>
__global__ __launch_bounds__(kThreads) void k_product_ifft_z(const float2* __restrict__ accs,
                                                             const double2* __restrict__ phase,
                                                             const float2* __restrict__ fa, float2* __restrict__ out,
                                                             const float2* __restrict__ twn) {
    constexpr int N = ColShape<M>::N, H = ColShape<M>::H;
    extern __shared__ float2 lds[];
    float2* a = lds;
    float2* twnl = a + N * COLS;
    const Blk b = xcd_block();
    const int c0 = b.x * COLS, iy = b.y, s = b.z;
    float2* dst = out + (size_t)s * N * N * H + (size_t)iy * H + c0;
    if (iy == N / 2) {
        for (int t = threadIdx.x; t < N * COLS; t += kThreads)
            dst[(size_t)(t / COLS) * N * H + t % COLS] = make_float2(0.f, 0.f);
        return;
    }
    load_table<N>(twnl, twn);
    const float2* src = accs + (size_t)s * N * N * H + (size_t)iy * H + c0;
    using P = RegPass<N, COLS>;
    float2 v[P::NBF][8];
#pragma unroll
    for (int u = 0; u < P::NBF; ++u) {
        const int t = u * kThreads + (int)threadIdx.x;
        if (P::WORK % kThreads == 0 || t < P::WORK) {
            const int cc = t % COLS, j = t / COLS;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int o = j + r * P::NB;
                const float2 acc = src[(size_t)o * N * H + cc];
                const float2 A = fa[((size_t)o * N + iy) * H + c0 + cc];
                v[u][r] = cmul(cmul(A, make_float2(acc.x, -acc.y)), shift_factor(phase, N, c0 + cc, iy, o));
            }
        }
    }
    fft_cols_regs<N, 1, COLS>(v, a, twnl);
    for (int t = threadIdx.x; t < N * COLS; t += kThreads) dst[(size_t)(t / COLS) * N * H + t % COLS] = a[t];
}

// a2 (z) for the lifted score: the z transform of each radius component kept
// apart, out [s][c][mz][my][mx], times the deconvolution if `deconv` is set
// (the fixed shape's component spectra) or plain (the rotated shape's, whose
// deconvolution is in the product's factor).  Same transforms, in the same
// order, as z_accumulate.
template <int M, int COLS>
__global__ __launch_bounds__(kThreads) void k_fft_z_components(const float2* __restrict__ in, int q,
                                                               const double* __restrict__ deconv,
                                                               float2* __restrict__ out,
                                                               const float2* __restrict__ twm,
                                                               const int* __restrict__ bin_start, int64_t nk, int w, int ygs) {
    constexpr int N = ColShape<M>::N, H = ColShape<M>::H;
    using P = RegPass<M, COLS>;
    extern __shared__ float2 lds[];
    __shared__ unsigned char zlive[M];
    float2* a = lds;
    float2* twl = a + M * COLS;
    const Blk b = xcd_block();
    const int c0 = b.x * COLS, iy = b.y, s = b.z;
    auto dst = [&](int c) { return out + (((size_t)s * q + c) * N * N) * H + (size_t)iy * H + c0; };
    if (iy == N / 2) {
        for (int c = 0; c < q; ++c)
            for (int t = threadIdx.x; t < N * COLS; t += kThreads)
                dst(c)[(size_t)(t / COLS) * N * H + t % COLS] = make_float2(0.f, 0.f);
        return;
    }
    load_table<M>(twl, twm);
    for (int t = threadIdx.x; t < M; t += kThreads)
        zlive[t] = zrow_live<M>(bin_start + (size_t)s * (SpreadShape<M>::KEYS + 1), nk, w, t, ygs);
    __syncthreads();
    for (int c = 0; c < q; ++c) {
        const float2* src = in + (((size_t)s * q + c) * M) * N * H + (size_t)iy * H + c0;
        float2 v[P::NBF][8];
#pragma unroll
        for (int u = 0; u < P::NBF; ++u) {
            const int t = u * kThreads + (int)threadIdx.x;
            if (P::WORK % kThreads == 0 || t < P::WORK) {
                const int cc = t % COLS, j = t / COLS;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int z = j + r * P::NB;
                    v[u][r] = zlive[z] ? src[(size_t)z * N * H + cc] : make_float2(0.f, 0.f);
                }
            }
        }
        fft_cols_regs_band<M, -1, COLS>(v, a, twl);
        float2* d = dst(c);
        for (int t = threadIdx.x; t < N * COLS; t += kThreads) {
            const int o = t / COLS, cc = t % COLS;
            const int si = kept_source<N, M>(o);
            float2 g = si < 0 ? make_float2(0.f, 0.f) : a[si * COLS + cc];
            if (deconv) {
                const float f = (float)(deconv[c0 + cc] * deconv[iy] * deconv[o]);
                g = make_float2(g.x * f, g.y * f);
            }
            d[(size_t)o * N * H + cc] = g;
        }
        __syncthreads();  // `a` is read out before the next component's pass
    }
}

// The fixed shape's side of one lifted slice: for every kept mode,
//   H[p'] = sum_p G_A[p] tab[p][p'][|m|^2]
// (G_A: its deconvolved component spectra), so that the slice's spectrum is
// sum_p' H[p'] conj(G_RB[p']) times the product's factor.  Arrays [c][mz][my][mx].
__global__ __launch_bounds__(kThreads) void k_lift_h(const float2* __restrict__ ga, int qa,
                                                     const float* __restrict__ tab, int qb, int m2n, int n,
                                                     float2* __restrict__ hh) {
    const int half = n / 2;
    const size_t modes = (size_t)n * n * half;
    const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= modes) return;
    const int mx = (int)(i % half), iy = (int)((i / half) % n), iz = (int)(i / ((size_t)half * n));
    const int my = iy < half ? iy : iy - n, mz = iz < half ? iz : iz - n;
    if (iy == half || iz == half) {
        for (int c = 0; c < qb; ++c) hh[(size_t)c * modes + i] = make_float2(0.f, 0.f);
        return;
    }
    const int m2 = mx * mx + my * my + mz * mz;
    float2 g[32];
    for (int p = 0; p < qa; ++p) g[p] = ga[(size_t)p * modes + i];
    for (int c = 0; c < qb; ++c) {
        float2 acc = make_float2(0.f, 0.f);
        for (int p = 0; p < qa; ++p) {
            const float t = tab[((size_t)p * qb + c) * m2n + m2];
            acc.x = fmaf(g[p].x, t, acc.x);
            acc.y = fmaf(g[p].y, t, acc.y);
        }
        hh[(size_t)c * modes + i] = acc;
    }
}

// a4 + inverse z of one lifted slice, from the rotated shape's component z
// sums comps [s][c][mz][my][mx]:
//   S = sum_c H[c] conj(comps[s][c]) * prod_d D(m_d) exp(i k_d o_d) / L,
// components summed in order, then the unnormalised inverse transform along z.
template <int M, int COLS>
__global__ __launch_bounds__(kThreads) void k_lift_product_ifft_z(const float2* __restrict__ comps, int q,
                                                                  const double2* __restrict__ phase,
                                                                  const float2* __restrict__ hh,
                                                                  float2* __restrict__ out,
                                                                  const float2* __restrict__ twn) {
    constexpr int N = ColShape<M>::N, H = ColShape<M>::H;
    extern __shared__ float2 lds[];
    float2* a = lds;
    float2* twnl = a + N * COLS;
    const Blk b = xcd_block();
    const int c0 = b.x * COLS, iy = b.y, s = b.z;
    float2* dst = out + (size_t)s * N * N * H + (size_t)iy * H + c0;
    if (iy == N / 2) {
        for (int t = threadIdx.x; t < N * COLS; t += kThreads)
            dst[(size_t)(t / COLS) * N * H + t % COLS] = make_float2(0.f, 0.f);
        return;
    }
    load_table<N>(twnl, twn);
    const size_t modes = (size_t)N * N * H;
    const float2* src = comps + (size_t)s * q * modes + (size_t)iy * H + c0;
    const float2* hs = hh + (size_t)iy * H + c0;
    using P = RegPass<N, COLS>;
    float2 v[P::NBF][8];
#pragma unroll
    for (int u = 0; u < P::NBF; ++u) {
        const int t = u * kThreads + (int)threadIdx.x;
        if (P::WORK % kThreads == 0 || t < P::WORK) {
            const int cc = t % COLS, j = t / COLS;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int o = j + r * P::NB;
                float2 acc = make_float2(0.f, 0.f);
                for (int c = 0; c < q; ++c) {
                    const float2 g = src[(size_t)c * modes + (size_t)o * N * H + cc];
                    const float2 hc = hs[(size_t)c * modes + (size_t)o * N * H + cc];
                    // hc * conj(g)
                    acc.x = fmaf(hc.x, g.x, fmaf(hc.y, g.y, acc.x));
                    acc.y = fmaf(hc.y, g.x, fmaf(-hc.x, g.y, acc.y));
                }
                v[u][r] = cmul(acc, shift_factor(phase, N, c0 + cc, iy, o));
            }
        }
    }
    fft_cols_regs<N, 1, COLS>(v, a, twnl);
    for (int t = threadIdx.x; t < N * COLS; t += kThreads) dst[(size_t)(t / COLS) * N * H + t % COLS] = a[t];
}

// a5: inverse y over [s][z][my][mx] -> [s][z][y][mx].  A workgroup reads all of
// its columns before it writes them back, so in == out (in place) is allowed.
template <int M, int COLS>
__global__ __launch_bounds__(kThreads) void k_ifft_y(const float2* in, float2* out, const float2* __restrict__ twn) {
    constexpr int N = ColShape<M>::N, H = ColShape<M>::H;
    extern __shared__ float2 lds[];
    float2* a = lds;
    float2* twl = a + N * COLS;
    load_table<N>(twl, twn);
    const int c0 = blockIdx.x * COLS;
    const size_t plane = (size_t)blockIdx.z * N + blockIdx.y;
    const float2* src = in + plane * N * H + c0;
    using P = RegPass<N, COLS>;
    float2 v[P::NBF][8];
#pragma unroll
    for (int u = 0; u < P::NBF; ++u) {
        const int t = u * kThreads + (int)threadIdx.x;
        if (P::WORK % kThreads == 0 || t < P::WORK) {
            const int c = t % COLS, j = t / COLS;
#pragma unroll
            for (int r = 0; r < 8; ++r) v[u][r] = src[(size_t)(j + r * P::NB) * H + c];
        }
    }
    fft_cols_regs<N, 1, COLS>(v, a, twl);
    float2* dst = out + plane * N * H + c0;
    for (int t = threadIdx.x; t < N * COLS; t += kThreads) dst[(size_t)(t / COLS) * H + t % COLS] = a[t];
}

// a5: inverse x, half-complex to real.  Two lines X1, X2 share one complex
// transform of Z = X1 + i X2 with both extended by Hermitian symmetry
// (X[n-m] = conj X[m], Nyquist 0, imaginary part of X[0] dropped); the real and
// imaginary parts of the result are the two score lines.  Each block also
// reduces its scores to (max, lowest index of the max) and, for the obstacle
// predicate (Sec. 3.1 eq. eq_obs), writes the bits score > thr of its points
// (bit b of word w: linear index 32 w + b) and counts them.
template <int M, int COLS>
__global__ __launch_bounds__(kThreads) void k_ifft_x(const float2* __restrict__ in, float* __restrict__ scores,
                                                     unsigned* __restrict__ mask, float thr,
                                                     float* __restrict__ pval, int* __restrict__ pidx,
                                                     int* __restrict__ pcnt, const float2* __restrict__ twn) {
    constexpr int N = ColShape<M>::N, H = ColShape<M>::H, SC = N + 1;
    // whole iterations of the output loop: every lane takes part in each ballot,
    // and a wave's 64 points are two whole mask words
    static_assert((2 * COLS * N) % kThreads == 0, "output loop must be whole");
    extern __shared__ float2 lds[];
    __shared__ float red_v[kThreads / 64];
    __shared__ int red_i[kThreads / 64];
    __shared__ int red_c[kThreads / 64];
    float2* a = lds;
    float2* twl = a + COLS * SC;
    load_table<N>(twl, twn);
    const int s = blockIdx.y;
    const size_t line0 = (size_t)blockIdx.x * 2 * COLS;
    const float2* src = in + (size_t)s * N * N * H + line0 * H;
    for (int t = threadIdx.x; t < COLS * N; t += kThreads) {
        const int c = t / N, mm = t % N;
        float2 z;
        if (mm == H) {
            z = make_float2(0.f, 0.f);
        } else {
            const bool lo = mm < H;
            const int mi = lo ? mm : N - mm;
            float2 x1 = src[(size_t)(2 * c) * H + mi];
            float2 x2 = src[(size_t)(2 * c + 1) * H + mi];
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
        a[c * SC + mm] = z;
    }
    __syncthreads();
    fft_cols<N, 1, COLS, true>(a, twl);
    const float2* res = a;
    float best = -INFINITY;
    int besti = 0x7fffffff;
    int cnt = 0;
    float* dst = scores ? scores + (size_t)s * N * N * N + line0 * N : nullptr;
    unsigned* mdst = mask ? mask + ((size_t)s * N * N * N + line0 * N) / 32 : nullptr;
    const int lane = threadIdx.x & 63;
    for (int t = threadIdx.x; t < 2 * COLS * N; t += kThreads) {
        const int l = t / N, x = t % N;
        const float2 zz = res[(l >> 1) * SC + x];
        const float v = (l & 1) ? zz.y : zz.x;
        if (dst) dst[(size_t)l * N + x] = v;
        const int gi = (int)((line0 + l) * N + x);
        if (v > best || (v == best && gi < besti)) {
            best = v;
            besti = gi;
        }
        const bool hit = v > thr;
        cnt += hit;
        if (mdst) {
            const unsigned long long b = __ballot(hit);
            if (lane == 0) {
                mdst[(t >> 5)] = (unsigned)b;
                mdst[(t >> 5) + 1] = (unsigned)(b >> 32);
            }
        }
    }
    // the largest value (lowest index among equals) and the count: within each
    // wave by lane shuffles, then over the waves; the result does not depend
    // on the order of the comparisons
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float v2 = __shfl_down(best, off, 64);
        const int i2 = __shfl_down(besti, off, 64);
        cnt += __shfl_down(cnt, off, 64);
        if (v2 > best || (v2 == best && i2 < besti)) {
            best = v2;
            besti = i2;
        }
    }
    const int wv = threadIdx.x >> 6;
    if (lane == 0) {
        red_v[wv] = best;
        red_i[wv] = besti;
        red_c[wv] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kThreads / 64; ++k) {
            if (red_v[k] > best || (red_v[k] == best && red_i[k] < besti)) {
                best = red_v[k];
                besti = red_i[k];
            }
            cnt += red_c[k];
        }
        pval[(size_t)s * gridDim.x + blockIdx.x] = best;
        pidx[(size_t)s * gridDim.x + blockIdx.x] = besti;
        if (pcnt) pcnt[(size_t)s * gridDim.x + blockIdx.x] = cnt;
    }
}

// Per rotation: the peak over the inverse-x blocks (out_val, out_idx; NULL: not
// wanted) and the obstacle count (out_cnt; NULL: not wanted).
__global__ __launch_bounds__(kThreads) void k_peak_final(const float* __restrict__ pval, const int* __restrict__ pidx,
                                                         const int* __restrict__ pcnt, int nblocks,
                                                         float* __restrict__ out_val, int64_t* __restrict__ out_idx,
                                                         int64_t* __restrict__ out_cnt) {
    constexpr int NWV = kThreads / 64;
    __shared__ float red_v[NWV];
    __shared__ int red_i[NWV];
    __shared__ long long red_c[NWV];
    const int s = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float best = -INFINITY;
    int besti = 0x7fffffff;
    long long cnt = 0;
    for (int t = threadIdx.x; t < nblocks; t += kThreads) {
        const float v = pval[(size_t)s * nblocks + t];
        const int i = pidx[(size_t)s * nblocks + t];
        if (v > best || (v == best && i < besti)) {
            best = v;
            besti = i;
        }
        if (out_cnt) cnt += pcnt[(size_t)s * nblocks + t];
    }
    // within each wave by lane shuffles, then over the waves (the largest value,
    // lowest index among equals, and the count do not depend on the order)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float v2 = __shfl_down(best, off, 64);
        const int i2 = __shfl_down(besti, off, 64);
        cnt += __shfl_down(cnt, off, 64);
        if (v2 > best || (v2 == best && i2 < besti)) {
            best = v2;
            besti = i2;
        }
    }
    if (lane == 0) {
        red_v[wv] = best;
        red_i[wv] = besti;
        red_c[wv] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < NWV; ++k) {
            if (red_v[k] > best || (red_v[k] == best && red_i[k] < besti)) {
                best = red_v[k];
                besti = red_i[k];
            }
            cnt += red_c[k];
        }
        if (out_cnt) out_cnt[s] = cnt;
        if (out_val) {
            out_val[s] = best;
            out_idx[s] = besti;
        }
    }
}

// ---------------------------------------------------------------------------
// Single-configuration query (Sec. 4.1, eq. eq_single): the score at arbitrary
// translations as the Parseval sum (1/L^3) sum_m F_A(k_m) conj(F_RB(k_m))
// exp(i k_m . t) over a truncated set of modes.  F_RB is evaluated directly at
// the kept modes (an NDFT of the rotated knots on the radius expansion), so no
// spreading grid is involved.  Modes are listed once per pair of +-m (half
// space: mx > 0, or mx = 0 and my > 0, or mx = my = 0 and mz >= 0); the
// summand of a pair is twice the real part of one of them, the DC once.
// ---------------------------------------------------------------------------
constexpr int kQBlock = 256;   // threads per workgroup
constexpr int kQModes = 64;    // modes per NDFT workgroup (a wave each), 4 knot groups
constexpr int kQMaxChunk = 256;

__device__ __forceinline__ void unpack_mode(int p, int& mx, int& my, int& mz) {
    mx = (p & 1023) - 512;
    my = ((p >> 10) & 1023) - 512;
    mz = ((p >> 20) & 1023) - 512;
}

// part[chunk][mode] = sum over the chunk's knots j of
//   (sum_c vtab[c][|m|^2] wts[c][j]) exp(-2 pi i m . (R y_j) / L);
// a workgroup takes kQModes modes, its four waves a quarter of the chunk each.
__global__ __launch_bounds__(kQBlock) void k_query_ndft(const int* __restrict__ modes, int nm,
                                                        const double* __restrict__ quat,
                                                        const double* __restrict__ pos,
                                                        const float* __restrict__ wts, int64_t nk, int q, int kch,
                                                        const float* __restrict__ vtab, int m2n, double inv_l,
                                                        float2* __restrict__ part) {
    __shared__ double su[kQMaxChunk][3];
    __shared__ float sw[32][kQMaxChunk];
    __shared__ float2 red[4][kQModes];
    const int chunk = blockIdx.y;
    const int64_t j0 = (int64_t)chunk * kch;
    const int nj = (int)min<int64_t>(kch, nk - j0);
    {
        const double nn = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
        const double w = quat[0] / nn, x = quat[1] / nn, y = quat[2] / nn, z = quat[3] / nn;
        const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),    2 * (x * z + w * y),
                             2 * (x * y + w * z),    1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                             2 * (x * z - w * y),    2 * (y * z + w * x),    1 - 2 * (x * x + y * y)};
        for (int t = threadIdx.x; t < nj; t += kQBlock) {
            const double px = pos[3 * (j0 + t)], py = pos[3 * (j0 + t) + 1], pz = pos[3 * (j0 + t) + 2];
            su[t][0] = (R[0] * px + R[1] * py + R[2] * pz) * inv_l;
            su[t][1] = (R[3] * px + R[4] * py + R[5] * pz) * inv_l;
            su[t][2] = (R[6] * px + R[7] * py + R[8] * pz) * inv_l;
            for (int c = 0; c < q; ++c) sw[c][t] = wts[(size_t)c * nk + j0 + t];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int mi = blockIdx.x * kQModes + lane;
    float ar = 0.f, ai = 0.f;
    if (mi < nm) {
        int mx, my, mz;
        unpack_mode(modes[mi], mx, my, mz);
        const int m2 = mx * mx + my * my + mz * mz;
        float v[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) v[c] = c < q ? vtab[(size_t)c * m2n + m2] : 0.f;
        for (int j = grp; j < nj; j += 4) {
            float kj = 0.f;
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                if (c >= q) break;
                kj += v[c] * sw[c][j];
            }
            // phase in cycles, reduced in FP64 before the FP32 sine and cosine
            const double ph = (double)mx * su[j][0] + (double)my * su[j][1] + (double)mz * su[j][2];
            const float f = (float)(ph - rint(ph));
            float sn, cs;
            sincospif(2.0f * f, &sn, &cs);
            ar += kj * cs;
            ai -= kj * sn;
        }
    }
    red[grp][lane] = make_float2(ar, ai);
    __syncthreads();
    if (grp == 0 && mi < nm) {
        const float2 a0 = red[0][lane], a1 = red[1][lane], a2 = red[2][lane], a3 = red[3][lane];
        part[(size_t)chunk * nm + mi] = make_float2((a0.x + a1.x) + (a2.x + a3.x), (a0.y + a1.y) + (a2.y + a3.y));
    }
}

// P[mode] = weight * F_A(k_m) conj(F_RB(k_m)) / L^3, F_RB = sum of the chunks in
// order; F_A from the prepared half spectrum [mz][my][mx], mx >= 0.
__global__ __launch_bounds__(kQBlock) void k_query_reduce(const int* __restrict__ modes, int nm, int chunks,
                                                          const float2* __restrict__ part,
                                                          const float2* __restrict__ fa, int n, double inv_l3,
                                                          float2* __restrict__ P) {
    const int mi = blockIdx.x * kQBlock + threadIdx.x;
    if (mi >= nm) return;
    float br = 0.f, bi = 0.f;
    for (int c = 0; c < chunks; ++c) {
        const float2 v = part[(size_t)c * nm + mi];
        br += v.x;
        bi += v.y;
    }
    int mx, my, mz;
    unpack_mode(modes[mi], mx, my, mz);
    const float2 A = fa[((size_t)((mz + n) % n) * n + (my + n) % n) * (n / 2) + mx];
    const float wgt = (float)(((mx | my | mz) == 0 ? 1.0 : 2.0) * inv_l3);
    // A * conj(B)
    P[mi] = make_float2((A.x * br + A.y * bi) * wgt, (A.y * br - A.x * bi) * wgt);
}

// tpart[t][b] = sum over mode block b of Re(P_m exp(2 pi i m . t / L)); the mode
// list is cut into gridDim.y blocks of mper modes.
__global__ __launch_bounds__(kQBlock) void k_query_sum(const int* __restrict__ modes, int nm, int mper,
                                                       const float2* __restrict__ P,
                                                       const double* __restrict__ t, double inv_l,
                                                       float* __restrict__ tpart) {
    __shared__ float red[kQBlock];
    const double tx = t[3 * blockIdx.x] * inv_l, ty = t[3 * blockIdx.x + 1] * inv_l, tz = t[3 * blockIdx.x + 2] * inv_l;
    const int m0 = blockIdx.y * mper, m1 = min(nm, m0 + mper);
    float acc = 0.f;
    for (int mi = m0 + threadIdx.x; mi < m1; mi += kQBlock) {
        int mx, my, mz;
        unpack_mode(modes[mi], mx, my, mz);
        const double ph = (double)mx * tx + (double)my * ty + (double)mz * tz;
        const float f = (float)(ph - rint(ph));
        float sn, cs;
        sincospif(2.0f * f, &sn, &cs);
        const float2 p = P[mi];
        acc += p.x * cs - p.y * sn;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kQBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) tpart[(size_t)blockIdx.x * gridDim.y + blockIdx.y] = red[0];
}

// out[t] = sum of its mode blocks, in order.
__global__ __launch_bounds__(kQBlock) void k_query_final(const float* __restrict__ tpart, int nb, int64_t n_t,
                                                         float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kQBlock + threadIdx.x;
    if (i >= n_t) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += tpart[(size_t)i * nb + b];
    out[i] = s;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

// Call f(std::integral_constant<int, M>) for the spreading-grid size m.
template <class F>
hipError_t with_m(int m, F&& f) {
    // f may return the error of a dispatch of its own (with_cols)
    auto call = [&](auto mc) -> hipError_t {
        if constexpr (std::is_same_v<decltype(f(mc)), hipError_t>) {
            return f(mc);
        } else {
            f(mc);
            return hipSuccess;
        }
    };
    hipError_t e;
    switch (m) {
        case 32: e = call(std::integral_constant<int, 32>{}); break;
        case 64: e = call(std::integral_constant<int, 64>{}); break;
        case 128: e = call(std::integral_constant<int, 128>{}); break;
        case 256: e = call(std::integral_constant<int, 256>{}); break;
        case 512: e = call(std::integral_constant<int, 512>{}); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// Call f(std::integral_constant<int, COLS>) for the width `want` (0: default)
// of a pass whose widths are C; an unlisted width is an error.
template <class C, class F>
hipError_t with_cols(int want, F&& f) {
    // f may return the error of a dispatch of its own (with_ty)
    auto call = [&](auto cc) -> hipError_t {
        if constexpr (std::is_same_v<decltype(f(cc)), hipError_t>) {
            return f(cc);
        } else {
            f(cc);
            return hipSuccess;
        }
    };
    if (want == 0 || want == C::DEF) return call(std::integral_constant<int, C::DEF>{});
    if (want == C::DN) return call(std::integral_constant<int, C::DN>{});
    if (want == C::UP) return call(std::integral_constant<int, C::UP>{});
    return hipErrorInvalidValue;
}

// two spreading workgroups per CU: dynamic LDS plus the kernel's static arrays
// must fit in half of the 160 KB
constexpr size_t kSpreadLds = 79 * 1024;

// bytes of one staged knot: component pair, cell, position, z weight, x and y weights
inline size_t staged_bytes(int w) { return 20 + 8 * (size_t)w; }

template <int M, int TYP>
int spread_cap_t(int w) {
    const size_t fixed = SpreadShape<M, TYP>::FIXED;
    const size_t room = fixed < kSpreadLds ? kSpreadLds - fixed : 0;
    int cap = (int)std::min<size_t>(512, room / staged_bytes(w));
    cap &= ~63;
    return cap < 64 ? 64 : cap;
}

template <int M, int TYP>
size_t spread_lds_t(int w) {
    return SpreadShape<M, TYP>::FIXED + (size_t)spread_cap_t<M, TYP>(w) * staged_bytes(w);
}

// Calls f with the spreading pass's tile height as a constant: the default at
// M, or half of it when the tuning chose that (tile_choices).
template <int M, class F>
auto with_ty(const Geom& g, F&& f) {
    constexpr int T0 = SpreadShape<M>::TY;
    if (g.tile_rows == T0 / 2) return f(std::integral_constant<int, T0 / 2>{});
    return f(std::integral_constant<int, T0>{});
}

}  // namespace

hipError_t launch_deconv_tables(const Geom& g, double box, const double origin[3], double* d_deconv,
                                double2* d_phase, hipStream_t st) {
    hipLaunchKernelGGL(k_deconv_tables, dim3((g.n + 127) / 128), dim3(128), 0, st, g.n, g.m, g.w,
                       (double)g.beta, box, origin[0], origin[1], origin[2], d_deconv, d_phase);
    return hipGetLastError();
}

hipError_t launch_ball_table(const Geom& g, double dk, const double* d_nodes, const double* d_basis, int p,
                             int q, double rref, double r0, double lam, float* d_vtab, hipStream_t st) {
    hipLaunchKernelGGL(k_ball_table, dim3((g.m2n + 127) / 128), dim3(128), 0, st, g.m2n, dk, d_nodes, d_basis,
                       p, q, rref, r0, lam, d_vtab);
    return hipGetLastError();
}

namespace {
int log2i(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}
int bin_blocks(int64_t nk) { return (int)((nk + kBinBlock - 1) / kBinBlock); }
}  // namespace

hipError_t launch_rotate_bin(const Geom& g, const double* d_quats, int S, const double* d_pos, int64_t nk,
                             int4* d_rec, int* d_rank, int* d_counts, int* d_bin_start, int* d_plan, hipStream_t st) {
    if (nk == 0 || S == 0) return hipSuccess;
    const int G = bin_group(g);
    hipLaunchKernelGGL(k_rotate_bin, dim3(bin_blocks(nk), S), dim3(kBinBlock), 0, st, d_quats, d_pos, nk, g.inv_hf,
                       g.m, log2i(G), g.m / G, bin_keys_max(g.m), d_rec, d_rank, d_counts, d_plan, plan_words());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_scan, dim3(S), dim3(kBinBlock), 0, st, d_counts, g.m * (g.m / G), bin_keys_max(g.m), nk,
                       d_bin_start);
    return hipGetLastError();
}

int plan_words() { return kPlanBuckets + 1; }

hipError_t launch_scatter_plan(const Geom& g, int S, int q, const Occupancy& occ, const int4* d_rec,
                               const float* d_wts, const int* d_rank, int* d_scell, float* d_skbw, float* d_swts,
                               int* d_plan, int* d_list, hipStream_t st) {
    if (occ.nk == 0 || S == 0) return hipSuccess;
    return with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        return with_ty<M>(g, [&](auto tc) {
            constexpr int TY = decltype(tc)::value;
            constexpr int tiles = M * (M / TY);
            const int G = bin_group(g);
            const int nscatter = bin_blocks(occ.nk);
            hipLaunchKernelGGL((k_scatter_plan<M, TY>), dim3(nscatter + (tiles + 255) / 256, S), dim3(256), 0, st,
                               d_rec, d_wts, d_rank, occ.bin_start, occ.nk, log2i(G), M / G, g.w, g.beta,
                               g.inv_i0beta, q, d_scell, d_skbw, d_swts, nscatter, occ.tile_live, d_plan, d_list,
                               S * tiles);
            return hipGetLastError();
        });
    });
}

size_t max_lds_bytes(const Geom& g, int qmax) {
    size_t need = 0;
    (void)with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        constexpr int N = M / 2;
        using C = ColShape<M>;
        constexpr int T0 = SpreadShape<M>::TY;
        need = std::max(need, std::max(spread_lds_t<M, T0>(g.w), spread_lds_t<M, T0 / 2>(g.w)));
        // the widest width of each pass
        need = std::max(need, sizeof(float2) * ((size_t)M * std::max(C::Y::UP, C::Z::UP) + M + N));
        need = std::max(need, sizeof(float2) * ((size_t)N * C::IY::UP + N));
        need = std::max(need, sizeof(float2) * ((size_t)C::IX::UP * (N + 1) + N) + 12 * kThreads);
    });
    return need;
}

int spread_tiles(const Geom& g) {
    int t = 0;
    (void)with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        with_ty<M>(g, [&](auto tc) { t = M / decltype(tc)::value; });
    });
    return t;
}

int spread_tiles_max(const Geom& g) {
    int t = 0;
    (void)with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        t = M / (SpreadShape<M>::TY / 2);
    });
    return t;
}

int tile_choices(int m, int out[2]) {
    int k = 0;
    (void)with_m(m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        out[k++] = SpreadShape<M>::TY;
        out[k++] = SpreadShape<M>::TY / 2;
    });
    return k;
}

hipError_t launch_spread_fftx(const Geom& g, int S, const Occupancy& occ, int* d_plan, const int* d_list,
                              const int* d_scell, const float* d_skbw, const float* d_swts, int q, float fix_scale,
                              float2* d_out, const float2* d_twm, unsigned long long* d_work, hipStream_t st) {
    if (S == 0 || occ.nk == 0) return hipSuccess;
    return with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        return with_ty<M>(g, [&](auto tc) {
            constexpr int TY = decltype(tc)::value;
            constexpr int tiles = M * (M / TY);
            hipLaunchKernelGGL((k_spread_fftx<M, TY>), dim3(std::max(1, g.spread_wgs)), dim3(kSpreadThreads),
                               (spread_lds_t<M, TY>(g.w)), st, occ.bin_start, occ.tile_live, d_plan, d_list,
                               S * tiles, d_scell, d_skbw, d_swts, occ.nk, q, g.w, (spread_cap_t<M, TY>(g.w)), fix_scale,
                               1.0f / fix_scale, d_out, d_twm, d_work,
                               (unsigned long long)occ.nk * S *
                                   (sizeof(int) + 3 * sizeof(float) * g.w + sizeof(float) * q),
                               log2i(bin_group(g)));
            return hipGetLastError();
        });
    });
}

// Fewest workgroups a y-pass grid is given when a row's components are split.
constexpr long kYMinBlocks = 16384;

hipError_t launch_fft_y(const Geom& g, int S, int q, const Occupancy& occ, const float2* d_in, float2* d_out,
                        const float2* d_twm, hipStream_t st) {
    if (S == 0 || q == 0) return hipSuccess;
    return with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        using C = ColShape<M>;
        return with_cols<typename C::Y>(g.cols_y, [&](auto cc) {
            constexpr int COLS = decltype(cc)::value;
            // components per workgroup: all of a row's, unless the grid would
            // then hold fewer than kYMinBlocks workgroups (one rotation of a
            // shape with many components needs them split to fill the chip)
            const long rows = (long)(C::H / COLS) * (M / C::YZB) * S;
            int cg = q;
            while (cg > 1 && rows * ((q + cg - 1) / cg) < kYMinBlocks) cg = (cg + 1) / 2;
            return with_ty<M>(g, [&](auto tc) {
                constexpr int TY = decltype(tc)::value;
                hipLaunchKernelGGL((k_fft_y<M, COLS, TY>), dim3(C::H / COLS, M / C::YZB, S * ((q + cg - 1) / cg)),
                                   dim3(kThreads), sizeof(float2) * ((size_t)M * COLS + M), st, d_in, d_out, d_twm,
                                   q, cg, occ.bin_start, occ.tile_live, occ.nk, g.w, log2i(bin_group(g)));
                return hipGetLastError();
            });
        });
    });
}

hipError_t launch_fft_z_spectrum(const Geom& g, const float2* d_in, int S, int q, const Occupancy& occ,
                                 const float* d_vtab, const double* d_deconv, float2* d_spec, const float2* d_twm,
                                 hipStream_t st) {
    return with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        using C = ColShape<M>;
        return with_cols<typename C::Z>(g.cols_z, [&](auto cc) {
            constexpr int COLS = decltype(cc)::value;
            hipLaunchKernelGGL((k_fft_z_spectrum<M, COLS>), dim3(C::H / COLS, C::N, S), dim3(kThreads),
                               sizeof(float2) * ((size_t)M * COLS + M), st, d_in, q, d_vtab, g.m2n, d_deconv,
                               d_spec, d_twm, occ.bin_start, occ.nk, g.w, log2i(bin_group(g)));
        });
    });
}

hipError_t launch_fft_z_product(const Geom& g, const float2* d_in, int S, int q, const Occupancy& occ,
                                const float* d_vtab, const double2* d_phase, const float2* d_fa, float2* d_out,
                                const float2* d_twm, const float2* d_twn, hipStream_t st) {
    return with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        using C = ColShape<M>;
        return with_cols<typename C::Z>(g.cols_z, [&](auto cc) {
            constexpr int COLS = decltype(cc)::value;
            hipLaunchKernelGGL((k_fft_z_product<M, COLS>), dim3(C::H / COLS, C::N, S), dim3(kThreads),
                               sizeof(float2) * ((size_t)M * COLS + M + C::N), st, d_in, q, d_vtab, g.m2n,
                               d_phase, d_fa, d_out, d_twm, d_twn, occ.bin_start, occ.nk, g.w,
                               log2i(bin_group(g)));
        });
    });
}

hipError_t launch_product_ifft_z(const Geom& g, const float2* d_acc, int S, const double2* d_phase,
                                 const float2* d_fa, float2* d_out, const float2* d_twn, hipStream_t st) {
    return with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        using C = ColShape<M>;
        return with_cols<typename C::IY>(g.cols_iy, [&](auto cc) {
            constexpr int COLS = decltype(cc)::value;
            hipLaunchKernelGGL((k_product_ifft_z<M, COLS>), dim3(C::H / COLS, C::N, S), dim3(kThreads),
                               sizeof(float2) * ((size_t)C::N * COLS + C::N), st, d_acc, d_phase, d_fa, d_out, d_twn);
        });
    });
}

hipError_t launch_lift_table(const Geom& g, double dk, const double* d_na, int qa, const double* d_nb, int qb,
                             double h, float* d_tab, hipStream_t st) {
    hipLaunchKernelGGL(k_lift_table, dim3((g.m2n + 127) / 128, qa * qb), dim3(128), 0, st, g.m2n, dk, d_na, qa, d_nb,
                       qb, h, d_tab);
    return hipGetLastError();
}

hipError_t launch_fft_z_components(const Geom& g, const float2* d_in, int S, int q, const Occupancy& occ,
                                   const double* d_deconv, float2* d_out, const float2* d_twm, hipStream_t st) {
    if (S == 0) return hipSuccess;
    return with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        using C = ColShape<M>;
        return with_cols<typename C::Z>(g.cols_z, [&](auto cc) {
            constexpr int COLS = decltype(cc)::value;
            hipLaunchKernelGGL((k_fft_z_components<M, COLS>), dim3(C::H / COLS, C::N, S), dim3(kThreads),
                               sizeof(float2) * ((size_t)M * COLS + M), st, d_in, q, d_deconv, d_out, d_twm,
                               occ.bin_start, occ.nk, g.w, log2i(bin_group(g)));
        });
    });
}

hipError_t launch_lift_h(const Geom& g, const float2* d_ga, int qa, const float* d_tab, int qb, float2* d_h,
                         hipStream_t st) {
    const size_t modes = (size_t)g.n * g.n * g.half;
    hipLaunchKernelGGL(k_lift_h, dim3((unsigned)((modes + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, d_ga, qa,
                       d_tab, qb, g.m2n, g.n, d_h);
    return hipGetLastError();
}

hipError_t launch_lift_product_ifft_z(const Geom& g, const float2* d_comps, int S, int q, const double2* d_phase,
                                      const float2* d_h, float2* d_out, const float2* d_twn, hipStream_t st) {
    return with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        using C = ColShape<M>;
        return with_cols<typename C::IY>(g.cols_iy, [&](auto cc) {
            constexpr int COLS = decltype(cc)::value;
            hipLaunchKernelGGL((k_lift_product_ifft_z<M, COLS>), dim3(C::H / COLS, C::N, S), dim3(kThreads),
                               sizeof(float2) * ((size_t)C::N * COLS + C::N), st, d_comps, q, d_phase, d_h, d_out,
                               d_twn);
        });
    });
}

hipError_t launch_ifft_y(const Geom& g, const float2* d_in, int S, float2* d_out, const float2* d_twn,
                         hipStream_t st) {
    return with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        using C = ColShape<M>;
        return with_cols<typename C::IY>(g.cols_iy, [&](auto cc) {
            constexpr int COLS = decltype(cc)::value;
            hipLaunchKernelGGL((k_ifft_y<M, COLS>), dim3(C::H / COLS, C::N, S), dim3(kThreads),
                               sizeof(float2) * ((size_t)C::N * COLS + C::N), st, d_in, d_out, d_twn);
        });
    });
}

int ifft_x_blocks(const Geom& g) {
    int nb = 0;
    (void)with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        using C = ColShape<M>;
        const int px = g.pairs_ix == 0 ? C::XCOLS : g.pairs_ix;
        nb = C::N * C::N / (2 * px);
    });
    return nb;
}

int ifft_x_blocks_max(const Geom& g) {
    int nb = 0;
    (void)with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        using C = ColShape<M>;
        nb = C::N * C::N / (2 * C::IX::DN);
    });
    return nb;
}

int bin_choices(int m, int out[3]) {
    const int g0 = bin_ygroup(m);
    int k = 0;
    out[k++] = g0;
    if (g0 > 1 && m * m / (g0 / 2) <= 32768) out[k++] = g0 / 2;
    if (2 * g0 <= m && m * m / (2 * g0) >= 1024) out[k++] = 2 * g0;
    return k;
}

int col_choices(int m, int pass, int out[3]) {
    int k = 0;
    (void)with_m(m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        using C = ColShape<M>;
        switch (pass) {
            case 0: k = C::Y::list(out); break;
            case 1: k = C::Z::list(out); break;
            case 2: k = C::IY::list(out); break;
            case 3: k = C::IX::list(out); break;
            default: k = 0;
        }
    });
    return k;
}

hipError_t launch_ifft_x(const Geom& g, const float2* d_in, int S, float* d_scores, unsigned* d_mask, float thr,
                         float* d_pval, int* d_pidx, int* d_pcnt, const float2* d_twn, hipStream_t st) {
    return with_m(g.m, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        using C = ColShape<M>;
        return with_cols<typename C::IX>(g.pairs_ix, [&](auto cc) {
            constexpr int COLS = decltype(cc)::value;
            hipLaunchKernelGGL((k_ifft_x<M, COLS>), dim3(C::N * C::N / (2 * COLS), S), dim3(kThreads),
                               sizeof(float2) * ((size_t)COLS * (C::N + 1) + C::N), st, d_in, d_scores, d_mask,
                               thr, d_pval, d_pidx, d_pcnt, d_twn);
        });
    });
}

hipError_t launch_peak_final(const float* d_pval, const int* d_pidx, const int* d_pcnt, int S, int nblocks,
                             float* d_peak_val, int64_t* d_peak_idx, int64_t* d_count, hipStream_t st) {
    hipLaunchKernelGGL(k_peak_final, dim3(S), dim3(kThreads), 0, st, d_pval, d_pidx, d_pcnt, nblocks, d_peak_val,
                       d_peak_idx, d_count);
    return hipGetLastError();
}

QueryPlan query_plan(int nm, int64_t nk, int64_t n_t) {
    QueryPlan p;
    const int mb = (nm + kQModes - 1) / kQModes;
    // knots per chunk: a power of two in 16..256, small enough for ~1024
    // workgroups, but at most 32 chunks (the reduction walks them in order)
    p.kch = kQMaxChunk;
    while (p.kch > 16 && (int64_t)mb * ((nk + p.kch - 1) / p.kch) < 1024 && (nk + p.kch / 2 - 1) / (p.kch / 2) <= 32)
        p.kch >>= 1;
    p.chunks = (int)std::max<int64_t>(1, (nk + p.kch - 1) / p.kch);
    // translation sums: enough mode blocks for ~1024 workgroups, at least 1024 modes each
    p.mblocks = 1;
    while (p.mblocks < 1024 && n_t * p.mblocks < 1024 && (int64_t)nm > 1024 * p.mblocks) p.mblocks <<= 1;
    p.mper = (nm + p.mblocks - 1) / p.mblocks;
    return p;
}

hipError_t launch_query(const Geom& g, const QueryPlan& qp, const int* d_modes, int nm, const double* d_quat,
                        const double* d_pos, const float* d_wts, int64_t nk, int q, const float* d_vtab, double box,
                        float2* d_part, const float2* d_fa, float2* d_P, const double* d_t, int64_t n_t,
                        float* d_tpart, float* d_out, hipStream_t st) {
    if (n_t == 0) return hipSuccess;
    if (nk > 0)  // an empty shape has F_RB = 0: the reduction below then sums no chunk
        hipLaunchKernelGGL(k_query_ndft, dim3((nm + kQModes - 1) / kQModes, qp.chunks), dim3(kQBlock), 0, st,
                           d_modes, nm, d_quat, d_pos, d_wts, nk, q, qp.kch, d_vtab, g.m2n, 1.0 / box, d_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_query_reduce, dim3((nm + kQBlock - 1) / kQBlock), dim3(kQBlock), 0, st, d_modes, nm,
                       nk > 0 ? qp.chunks : 0, d_part, d_fa, g.n, 1.0 / (box * box * box), d_P);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_query_sum, dim3((unsigned)n_t, qp.mblocks), dim3(kQBlock), 0, st, d_modes, nm, qp.mper,
                       d_P, d_t, 1.0 / box, d_tpart);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_query_final, dim3((unsigned)((n_t + kQBlock - 1) / kQBlock)), dim3(kQBlock), 0, st,
                       d_tpart, qp.mblocks, n_t, d_out);
    return hipGetLastError();
}

}  // namespace corr


// Host side of libcorr: the C ABI of include/corr.h, input validation, planning
// (window, grids, radius expansion), device memory and the stage sequence.
#include "corr.h"
#include "corr_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using corr::Geom;

namespace {

thread_local std::string g_thread_error = "no error";

struct CorrError {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw CorrError{code, buf};
}

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? CORR_ENOMEM : CORR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Radius expansion of the ball transform.
//
// Bhat(k; r) = (4 pi / 3) r^3 Phi(k r), Phi(x) = 3 (sin x - x cos x) / x^3.  Over
// the radii of one shape, f(k, r) = (r / rhi)^3 Phi(k r) is interpolated in r at
// p Chebyshev points r_b (barycentric basis l_b), and the interpolant is
// compressed onto the q leading right singular vectors V of the matrix
// f(k_a, r_b) over the needed wavenumbers.  Then
//     Bhat(k; r) ~ (4 pi / 3) rhi^3 sum_c [ sum_b f(k, r_b) V_bc ] [ sum_b l_b(r) V_bc ]
// so every knot spreads q weights c_i u_c(r_i) and the spectrum is the sum of
// the q component spectra times the k-factors.  q is the smallest count whose
// error max |f - approx| over the wavenumbers and a dense set of radii is <= tol.
// Equal radii give q = 1 exactly.
// ---------------------------------------------------------------------------
double ball_shape_host(double x) {
    if (x < 0.5) {
        double x2 = x * x;
        return 3.0 * (1.0 / 3.0 - x2 * (1.0 / 30.0 - x2 * (1.0 / 840.0 - x2 * (1.0 / 45360.0 - x2 * (1.0 / 3991680.0 - x2 * (1.0 / 518918400.0))))));
    }
    return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

// Separable expansion K(k; r) ~ (4 pi / 3) rref^3 sum_c v_c(k) u_c(r) of the per-ball
// kernel K(k; r) = Bhat(k; r + r0) - lam Bhat(k; r) over the radius range
// [rlo, rhi]; r0 = lam = 0 is the ball transform.
struct Expansion {
    int p = 1, q = 1;
    double rlo = 1, rhi = 1, err = 0;
    double r0 = 0, lam = 0, rref = 1;  // kernel parameters; rref = rhi + r0
    std::vector<double> nodes;  // [p]
    std::vector<double> basis;  // [p][q]
    std::vector<double> bary;   // barycentric weights [p]
};

// barycentric Lagrange basis l_b(r) at the nodes
void lagrange_row(const Expansion& e, double r, double* out) {
    for (int b = 0; b < e.p; ++b)
        if (r == e.nodes[b]) {
            for (int j = 0; j < e.p; ++j) out[j] = (j == b) ? 1.0 : 0.0;
            return;
        }
    double s = 0;
    for (int b = 0; b < e.p; ++b) {
        out[b] = e.bary[b] / (r - e.nodes[b]);
        s += out[b];
    }
    for (int b = 0; b < e.p; ++b) out[b] /= s;
}

// cyclic Jacobi eigen-decomposition of a symmetric p x p matrix (row-major);
// on return a's diagonal holds the eigenvalues and v the eigenvectors (columns).
void jacobi_eig(std::vector<double>& a, std::vector<double>& v, int p) {
    v.assign((size_t)p * p, 0.0);
    for (int i = 0; i < p; ++i) v[(size_t)i * p + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0, tot = 0;
        for (int i = 0; i < p; ++i)
            for (int j = 0; j < p; ++j) {
                double x = a[(size_t)i * p + j] * a[(size_t)i * p + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-30 * tot) break;
        for (int i = 0; i < p - 1; ++i)
            for (int j = i + 1; j < p; ++j) {
                double aij = a[(size_t)i * p + j];
                if (std::fabs(aij) < 1e-300) continue;
                double aii = a[(size_t)i * p + i], ajj = a[(size_t)j * p + j];
                double theta = (ajj - aii) / (2.0 * aij);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < p; ++k) {
                    double aki = a[(size_t)k * p + i], akj = a[(size_t)k * p + j];
                    a[(size_t)k * p + i] = c * aki - s * akj;
                    a[(size_t)k * p + j] = s * aki + c * akj;
                }
                for (int k = 0; k < p; ++k) {
                    double aik = a[(size_t)i * p + k], ajk = a[(size_t)j * p + k];
                    a[(size_t)i * p + k] = c * aik - s * ajk;
                    a[(size_t)j * p + k] = s * aik + c * ajk;
                }
                for (int k = 0; k < p; ++k) {
                    double vki = v[(size_t)k * p + i], vkj = v[(size_t)k * p + j];
                    v[(size_t)k * p + i] = c * vki - s * vkj;
                    v[(size_t)k * p + j] = s * vki + c * vkj;
                }
            }
    }
}

Expansion build_expansion(double rlo, double rhi, double dk, int m2n, double tol, double r0, double lam) {
    Expansion e;
    e.rlo = rlo;
    e.rhi = rhi;
    e.r0 = r0;
    e.lam = lam;
    e.rref = rhi + r0;
    // the kernel normalised by (4 pi / 3) rref^3
    auto f = [&](double k, double r) {
        const double rg = (r + r0) / e.rref, rr = r / e.rref;
        double v = rg * rg * rg * ball_shape_host(k * (r + r0));
        if (lam != 0.0) v -= lam * rr * rr * rr * ball_shape_host(k * r);
        return v;
    };
    if (!(rhi > rlo * (1.0 + 1e-12))) {
        e.p = e.q = 1;
        e.nodes = {rhi};
        e.basis = {1.0};
        e.bary = {1.0};
        // radii within 1e-12 relative: the error is that of using rhi for all
        double kmax = dk * std::sqrt((double)(m2n - 1));
        double worst = 0;
        for (int a = 0; a < 257; ++a) {
            double k = kmax * a / 256.0;
            worst = std::max(worst, std::fabs(f(k, rlo) - f(k, rhi)));
        }
        e.err = worst;
        return e;
    }
    const int p = 64;
    e.p = p;
    e.nodes.resize(p);
    e.bary.resize(p);
    for (int b = 0; b < p; ++b) {  // Chebyshev extreme points, barycentric weights (-1)^b, halved at the ends
        e.nodes[b] = 0.5 * (rlo + rhi) + 0.5 * (rhi - rlo) * std::cos(M_PI * b / (p - 1));
        e.bary[b] = ((b % 2) ? -1.0 : 1.0) * ((b == 0 || b == p - 1) ? 0.5 : 1.0);
    }
    // rows: every |m|^2 (all needed wavenumbers)
    std::vector<double> F((size_t)m2n * p);
    for (int a = 0; a < m2n; ++a) {
        double k = dk * std::sqrt((double)a);
        for (int b = 0; b < p; ++b) F[(size_t)a * p + b] = f(k, e.nodes[b]);
    }
    std::vector<double> G((size_t)p * p, 0.0);
    for (int a = 0; a < m2n; ++a) {
        const double* row = &F[(size_t)a * p];
        for (int i = 0; i < p; ++i)
            for (int j = i; j < p; ++j) G[(size_t)i * p + j] += row[i] * row[j];
    }
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < i; ++j) G[(size_t)i * p + j] = G[(size_t)j * p + i];
    std::vector<double> V;
    jacobi_eig(G, V, p);
    std::vector<int> order(p);
    for (int i = 0; i < p; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return G[(size_t)x * p + x] > G[(size_t)y * p + y]; });
    // test radii: the nodes, the midpoints between them and the ends
    std::vector<double> rt;
    for (int b = 0; b < p; ++b) rt.push_back(e.nodes[b]);
    for (int b = 0; b + 1 < p; ++b) rt.push_back(0.5 * (e.nodes[b] + e.nodes[b + 1]));
    const int nt = (int)rt.size();
    std::vector<double> L((size_t)nt * p);
    for (int t = 0; t < nt; ++t) lagrange_row(e, rt[t], &L[(size_t)t * p]);
    // residual over (wavenumber, test radius); rows sub-sampled for speed, then
    // the chosen q is re-checked on every row
    std::vector<double> resid((size_t)m2n * nt);
    for (int a = 0; a < m2n; ++a) {
        double k = dk * std::sqrt((double)a);
        for (int t = 0; t < nt; ++t) resid[(size_t)a * nt + t] = f(k, rt[t]);
    }
    std::vector<double> chosen;  // p x q, column-major build
    int q = 0;
    double err = 0;
    std::vector<double> kf(m2n), uf(nt);
    while (q < std::min(p, 32)) {
        int col = order[q];
        for (int a = 0; a < m2n; ++a) {
            double s = 0;
            for (int b = 0; b < p; ++b) s += F[(size_t)a * p + b] * V[(size_t)b * p + col];
            kf[a] = s;
        }
        for (int t = 0; t < nt; ++t) {
            double s = 0;
            for (int b = 0; b < p; ++b) s += L[(size_t)t * p + b] * V[(size_t)b * p + col];
            uf[t] = s;
        }
        err = 0;
        for (int a = 0; a < m2n; ++a)
            for (int t = 0; t < nt; ++t) {
                double& r = resid[(size_t)a * nt + t];
                r -= kf[a] * uf[t];
                err = std::max(err, std::fabs(r));
            }
        for (int b = 0; b < p; ++b) chosen.push_back(V[(size_t)b * p + col]);
        ++q;
        if (err <= tol) break;
    }
    if (err > tol) fail(CORR_EUNSUPPORTED, "radius expansion reaches only %.3g (tolerance %.3g) with 32 components; radii span [%g, %g]",
                        err, tol, rlo, rhi);
    e.q = q;
    e.err = err;
    e.basis.assign((size_t)p * q, 0.0);
    for (int c = 0; c < q; ++c)
        for (int b = 0; b < p; ++b) e.basis[(size_t)b * q + c] = chosen[(size_t)c * p + b];
    return e;
}

// ---------------------------------------------------------------------------
// Radius expansion of the lifted kernel (CORR_LIFTED_SCORE).  A pair's kernel
// What(k; r_i + rho_j - h) depends on both radii through their sum; it is
// interpolated in each radius at Chebyshev points of that shape's radius
// range,
//     What(k; r + rho - h) ~ sum_p sum_p' l_p(r) l'_p'(rho) What(k; a_p + b_p' - h),
// so each knot spreads its weight times the Lagrange basis l_p(r_i) (q = the
// node count) and the node-pair table What(k; a_p + b_p' - h) joins the two
// shapes' component spectra per slice height.  The node count is the smallest
// (2..32) whose interpolation error in this shape's radius, over 48
// wavenumbers up to the largest kept one, the other shape's radius range and
// the planned heights, is within tol of the largest kernel value.
// ---------------------------------------------------------------------------
// 3D transform of the 4D cone-intersection volume pi (P^2 - d^2)^2 / 24 (x = kP;
// Taylor series below x = 2, where the closed form cancels to x^7).
double lift_what_host(double k, double P) {
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
    const double k2 = k * k, k7 = k2 * k2 * k2 * k;
    return 4.0 * M_PI * M_PI * (x * x * x * std::cos(x) - 6.0 * x * x * std::sin(x) - 15.0 * x * std::cos(x) +
                                15.0 * std::sin(x)) / (3.0 * k7);
}

Expansion build_lift_expansion(double lo, double hi, double olo, double ohi, double hlo, double hhi, double dk,
                               int m2n, double tol) {
    Expansion e;
    e.rlo = lo;
    e.rhi = hi;
    e.rref = hi;
    const double kmax = dk * std::sqrt((double)(m2n - 1));
    const double scale = lift_what_host(0.0, hi + ohi - hlo);
    double ks[48], bs[5];
    for (int a = 0; a < 48; ++a) ks[a] = kmax * a / 47.0;
    for (int b = 0; b < 5; ++b) bs[b] = olo + (ohi - olo) * b / 4.0;
    const double hs[3] = {hlo, std::min(std::max(0.0, hlo), hhi), hhi};
    if (!(hi > lo * (1.0 + 1e-12))) {
        e.p = e.q = 1;
        e.nodes = {hi};
        e.basis = {1.0};
        e.bary = {1.0};
        double worst = 0;
        for (double k : ks)
            for (double b : bs)
                for (double h : hs) worst = std::max(worst, std::fabs(lift_what_host(k, lo + b - h) - lift_what_host(k, hi + b - h)));
        e.err = worst / scale;
        return e;
    }
    std::vector<double> lrow, f;
    for (int p = 2; p <= 32; ++p) {
        e.p = p;
        e.nodes.resize(p);
        e.bary.resize(p);
        for (int b = 0; b < p; ++b) {
            e.nodes[b] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * std::cos(M_PI * b / (p - 1));
            e.bary[b] = ((b % 2) ? -1.0 : 1.0) * ((b == 0 || b == p - 1) ? 0.5 : 1.0);
        }
        const int nt = 4 * p;
        std::vector<std::vector<double>> L(nt, std::vector<double>(p));
        std::vector<double> rt(nt);
        for (int t = 0; t < nt; ++t) {
            rt[t] = lo + (hi - lo) * (t + 0.5) / nt;
            lagrange_row(e, rt[t], L[t].data());
        }
        double err = 0;
        f.resize(p);
        for (double k : ks)
            for (double b : bs)
                for (double h : hs) {
                    for (int q = 0; q < p; ++q) f[q] = lift_what_host(k, e.nodes[q] + b - h);
                    for (int t = 0; t < nt; ++t) {
                        double v = 0;
                        for (int q = 0; q < p; ++q) v += L[t][q] * f[q];
                        err = std::max(err, std::fabs(v - lift_what_host(k, rt[t] + b - h)));
                    }
                }
        e.err = err / scale;
        if (e.err <= tol) {
            e.q = p;
            e.basis.assign((size_t)p * p, 0.0);
            for (int b = 0; b < p; ++b) e.basis[(size_t)b * p + b] = 1.0;
            return e;
        }
    }
    fail(CORR_EUNSUPPORTED, "lifted kernel: 32 radius nodes reach only %.3g (tolerance %.3g); radii span [%g, %g]",
         e.err, tol, lo, hi);
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
struct DevMem {
    std::vector<void*> ptrs;
    size_t bytes = 0;
    template <class T>
    T* alloc(size_t count) {
        if (count == 0) count = 1;
        size_t nb = count * sizeof(T);
        if (const char* cap = std::getenv("CORR_TEST_MAX_BYTES")) {
            if (bytes + nb > (size_t)std::strtoull(cap, nullptr, 10))
                fail(CORR_ENOMEM, "device allocation of %zu bytes exceeds the CORR_TEST_MAX_BYTES cap", nb);
        }
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, nb);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(CORR_ENOMEM, "hipMalloc(%zu): %s", nb, hipGetErrorString(e));
        }
        ptrs.push_back(p);
        bytes += nb;
        return static_cast<T*>(p);
    }
    void release() {
        for (void* p : ptrs) (void)hipFree(p);
        ptrs.clear();
        bytes = 0;
    }
};

struct Shape {
    int64_t n = 0;
    Expansion ex;
    float fix_scale = 1.0f;  // fixed-point scale of the spreading sums
    double* pos = nullptr;  // [n][3]
    float* wts = nullptr;   // [q][n]
    float* vtab = nullptr;  // [q][m2n]
    double* d_nodes = nullptr;  // [p] radius nodes of the expansion (device)
    double* rad = nullptr;      // [n] radii (device; the rasterization baseline)
};

// One offset slice: A's balls with every radius changed by delta, and its spectrum.
struct Slice {
    double delta = 0;
    Shape A;
    float2* fa = nullptr;  // [n][n][half]
};

}  // namespace

namespace corr {

// Buffers of one pipeline pass, `slots` rotations at a time; every per-slot
// region is sized for the largest plan that uses the workspace.
struct WsReq {
    size_t buf0 = 0, buf1 = 0;      // floats, float2 per slot
    size_t nk = 1, nkw = 1, nkq = 1;  // knots, knots*3w, knots*q per slot
    size_t counts = 1, bins = 1;    // sort keys, keys + 1 per slot
    size_t blocks = 1;              // inverse-x blocks per slot
    size_t tiles = 1;               // spreading tiles (m z rows x y tiles) per slot
    size_t list = 1;                // live-tile list entries per slot
    void merge(const WsReq& o) {
        buf0 = std::max(buf0, o.buf0); buf1 = std::max(buf1, o.buf1);
        nk = std::max(nk, o.nk); nkw = std::max(nkw, o.nkw); nkq = std::max(nkq, o.nkq);
        counts = std::max(counts, o.counts); bins = std::max(bins, o.bins); blocks = std::max(blocks, o.blocks);
        tiles = std::max(tiles, o.tiles);
        list = std::max(list, o.list);
    }
    // The request of k slots, as one slot.
    WsReq scaled(size_t k) const {
        WsReq o = *this;
        o.buf0 *= k; o.buf1 *= k; o.nk *= k; o.nkw *= k; o.nkq *= k;
        o.counts *= k; o.bins *= k; o.blocks *= k; o.tiles *= k; o.list *= k;
        return o;
    }
    // Rotations per pass that fit, for a plan needing `o` per slot, in buffers
    // sized for `slots` slots of this request (each array is indexed by the
    // plan's own geometry, so a smaller plan packs more rotations into them).
    int slots_for(const WsReq& o, int slots) const {
        size_t fit = 256;
        const size_t have[10] = {buf0, buf1, nk, nkw, nkq, counts, bins, blocks, tiles, list};
        const size_t need[10] = {o.buf0, o.buf1, o.nk, o.nkw, o.nkq, o.counts, o.bins, o.blocks, o.tiles, o.list};
        for (int k = 0; k < 10; ++k) fit = std::min(fit, (size_t)slots * have[k] / std::max<size_t>(need[k], 1));
        return (int)std::max<size_t>(fit, 1);
    }
    // device bytes of one slot: the arrays of Workspace below, element by element
    size_t slot_bytes() const {
        return 4 * buf0 + 8 * buf1 + 16 * nk /*rec*/ + 8 * nk /*rank, scell*/ + 4 * nkw /*skbw*/ + 4 * nkq /*swts*/ +
               4 * (counts + bins) + 12 * blocks + tiles + 4 * list + 32 /*quats*/;
    }
};

struct Workspace {
    int slots = 1;
    WsReq req;
    DevMem mem;
    float* buf0 = nullptr;         // [slots][q][m][n][half] complex (after y; reused after inverse z)
    float2* buf1 = nullptr;        // [slots][q][m^2][half] (after spread + x; reused after product)
    int4* rec = nullptr;           // [slots][nk] packed cell of each knot and its offsets from it (FP32 bits)
    int* rank = nullptr;           // [slots][nk] rank among the knots of its sort key
    int* counts = nullptr;         // [slots][keys] knots per sort key; zero between passes
    int* bin_start = nullptr;      // [slots][keys + 1] first sorted knot of each key
    unsigned char* tile_live = nullptr;  // [slots][m][y tiles] spreading tiles that some knot reaches
    int* plan = nullptr;           // bucket sizes and work counter of the spreading pass's live-tile plan
    unsigned long long* work = nullptr;  // [3] spreading work since the last read (corr_spread_work)
    int* list = nullptr;           // [buckets][slots * tiles] live tiles
    int* scell = nullptr;          // [slots][nk] sorted by z-cell: packed cell
    float* skbw = nullptr;         // [slots][nk][3][w]              window weights
    float* swts = nullptr;         // [slots][nk][q]                 component weights
    double* quats = nullptr;       // [slots][4]
    float* pval = nullptr;         // [slots][blocks] inverse-x block peaks
    int* pidx = nullptr;
    int* pcnt = nullptr;           // [slots][blocks] inverse-x block obstacle counts
    double* host_quats = nullptr;  // pinned [slots][4]
    hipEvent_t quat_done = nullptr;

    // qslots: rotations the staging of quaternions must hold (at least nslots)
    void allocate(int nslots, const WsReq& r, hipStream_t st, int qslots = 0) {
        slots = nslots;
        req = r;
        const size_t S = (size_t)nslots;
        const size_t SQ = (size_t)std::max(nslots, qslots);
        buf0 = mem.alloc<float>(S * r.buf0);
        buf1 = mem.alloc<float2>(S * r.buf1);
        rec = mem.alloc<int4>(S * r.nk);
        rank = mem.alloc<int>(S * r.nk);
        counts = mem.alloc<int>(S * r.counts);
        // the sort's counters start at zero; every scan clears them again
        hip_check(hipMemsetAsync(counts, 0, sizeof(int) * S * r.counts, st), "hipMemsetAsync");
        bin_start = mem.alloc<int>(S * r.bins);
        tile_live = mem.alloc<unsigned char>(S * r.tiles);
        plan = mem.alloc<int>(corr::plan_words());
        work = mem.alloc<unsigned long long>(3);
        hip_check(hipMemsetAsync(work, 0, 3 * sizeof(unsigned long long), st), "hipMemsetAsync");
        list = mem.alloc<int>(S * r.list);
        scell = mem.alloc<int>(S * r.nk);
        skbw = mem.alloc<float>(S * r.nkw);
        swts = mem.alloc<float>(S * r.nkq);
        quats = mem.alloc<double>(SQ * 4);
        pval = mem.alloc<float>(S * r.blocks);
        pidx = mem.alloc<int>(S * r.blocks);
        pcnt = mem.alloc<int>(S * r.blocks);
        hip_check(hipHostMalloc((void**)&host_quats, sizeof(double) * 4 * SQ, hipHostMallocDefault), "hipHostMalloc");
        hip_check(hipEventCreateWithFlags(&quat_done, hipEventDisableTiming), "hipEventCreate");
        hip_check(hipEventRecord(quat_done, st), "event");
    }
    void release() {
        mem.release();
        if (host_quats) (void)hipHostFree(host_quats);
        host_quats = nullptr;
        if (quat_done) (void)hipEventDestroy(quat_done);
        quat_done = nullptr;
    }
};

}  // namespace corr

// Graph replay of whole evaluations: every launch of one corr_eval (or
// corr_batch_eval) call, all batches of rotations, is captured once on a
// private stream and replayed by one hipGraphLaunch on the caller's stream as
// long as the call's device pointers, sizes and launch shapes stay the same
// (`key`).  The rotations are the only per-call input the graph reads: they
// are copied into a device array of fixed address before each launch.
struct GraphState {
    hipStream_t cap = nullptr;      // capture stream (default priority)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> key;      // what `exec` was captured for
    double* d_quats = nullptr;      // device [cap_rot][4]
    double* h_quats = nullptr;      // pinned [cap_rot][4]
    int64_t cap_rot = 0;
    hipEvent_t copied = nullptr;    // the last copy out of h_quats
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        key.clear();
    }
    void release() {
        drop_graph();
        if (d_quats) (void)hipFree(d_quats);
        if (h_quats) (void)hipHostFree(h_quats);
        if (copied) (void)hipEventDestroy(copied);
        if (cap) (void)hipStreamDestroy(cap);
        d_quats = nullptr;
        h_quats = nullptr;
        copied = nullptr;
        cap = nullptr;
        cap_rot = 0;
    }
};

struct corr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Geom g;
    double box = 0, origin[3] = {0, 0, 0}, sigma = 2, tol = 1e-6;
    double sc_r0 = 0, sc_lam = 0;  // shape-complementarity kernel parameters (0, 0: overlap score)
    bool lifted = false;           // CORR_LIFTED_SCORE: slices of the lifted correlation
    double lift_lo = 0, lift_hi = 0;  // allowed slice heights
    float* lift_tab = nullptr;     // [q_A][q_B][m2n] node-pair kernel table of one height
    float2* lift_ga = nullptr;     // [q_A][n][n][half] A's deconvolved component spectra
    uint32_t flags = 0;
    bool graph = false;       // replay evaluations as captured hipGraphs (corr_set_tuning)
    uint64_t shape_gen = 0;   // bumped whenever launch shapes, workspace or slices change
    GraphState gs;
    int qmax = 1;
    int64_t nkmax = 1;  // max(nA, nB, 1)
    Shape A, B;
    std::vector<corr_ball> host_a;  // A as given (offset slices are planned from it)
    std::vector<Slice> slices;      // corr_set_offsets
    DevMem slice_mem;
    DevMem mem;
    float2 *twm = nullptr, *twn = nullptr;
    double* deconv = nullptr;
    double2* phase = nullptr;
    float2* fa = nullptr;          // fixed shape's spectrum [n][n][half]
    double* ident_q = nullptr;     // the identity quaternion (1, 0, 0, 0), device
    corr::Workspace* ws = nullptr;  // per-rotation buffers (shared by the pairs of a batch)
    bool own_ws = false;
    int slots_eff = 0;  // rotations per pass of a batch pair (0: the workspace's slots)
    // A's spectrum on a side stream (contexts with a workspace of their own):
    // forked from `stream`, with buffers of its own, joined back by a_done
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, a_done = nullptr;
    bool a_pending = false;          // a_done not yet waited for on `stream`
    corr::Workspace* ws_a = nullptr;
    corr::Workspace* last_ws = nullptr;  // buffers of the last spreading pass
    // the last spreading pass: rotations, components, knots
    int last_S = 0, last_q = 0;
    int64_t last_nk = 0;
    // single-configuration query: half-space mode list of the last radius, and
    // buffers grown on demand (freed at destroy or when they grow)
    struct Grown {
        void* p = nullptr;
        size_t cap = 0;
    };
    Grown q_modes, q_part, q_P, q_t, q_quat, q_tpart;
    Grown r_grid, r_tw, r_quat;  // rasterization baseline: sample grid, FP64 twiddles, rotations
    double* q_host = nullptr;  // pinned staging of the rotation and translations
    size_t q_host_cap = 0;
    hipEvent_t q_done = nullptr;  // the last copy out of q_host
    int32_t q_r2 = -1;
    int q_nm = 0;
    int64_t q_full = 0;
    // stage timing (corr_profile): event pairs recorded around each launch
    bool profiling = false;
    struct Mark { int stage; hipEvent_t a, b; };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> spare;
    std::string err = "no error";
};

namespace {


void upload(void* dst, const void* src, size_t bytes, hipStream_t st) {
    hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st), "hipMemcpyAsync H2D");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

void validate_balls(const corr_ball* p, int64_t n, const char* name) {
    if (n < 0) fail(CORR_EINVAL, "%s: negative ball count %lld", name, (long long)n);
    if (n > 0 && !p) fail(CORR_EINVAL, "%s: NULL ball array with count %lld", name, (long long)n);
    if (n > (int64_t)1 << 31) fail(CORR_EUNSUPPORTED, "%s: more than 2^31 balls", name);
    for (int64_t i = 0; i < n; ++i) {
        const corr_ball& b = p[i];
        if (!std::isfinite(b.x) || !std::isfinite(b.y) || !std::isfinite(b.z))
            fail(CORR_EINVAL, "%s[%lld]: non-finite centre", name, (long long)i);
        if (!std::isfinite(b.r) || !(b.r > 0)) fail(CORR_EINVAL, "%s[%lld]: radius must be finite and > 0", name, (long long)i);
        if (!std::isfinite(b.w)) fail(CORR_EINVAL, "%s[%lld]: non-finite weight", name, (long long)i);
    }
}

// Smallest and largest radius (1, 1 for an empty set).
void radius_range(const corr_ball* balls, int64_t n, double& rlo, double& rhi) {
    rlo = rhi = 1.0;
    if (n > 0) {
        rlo = rhi = balls[0].r;
        for (int64_t i = 1; i < n; ++i) {
            rlo = std::min(rlo, balls[i].r);
            rhi = std::max(rhi, balls[i].r);
        }
    }
}

// Plan shape s's radius expansion; a lifted score also needs the other
// shape's balls (its kernel depends on both radii).
void setup_shape(corr_ctx* c, Shape& s, const corr_ball* balls, int64_t n, double dk,
                 const corr_ball* other = nullptr, int64_t n_other = 0) {
    s.n = n;
    double rlo, rhi;
    radius_range(balls, n, rlo, rhi);
    if (c->lifted) {
        double olo, ohi;
        radius_range(other, n_other, olo, ohi);
        s.ex = build_lift_expansion(rlo, rhi, olo, ohi, c->lift_lo, c->lift_hi, dk, c->g.m2n, c->tol);
        return;
    }
    s.ex = build_expansion(rlo, rhi, dk, c->g.m2n, c->tol, c->sc_r0, c->sc_lam);
}

// Storage order of a shape's balls on the device: Morton order of their
// centres (10 bits per axis over the centres' bounding box, ties by index).
// Balls near in space are then near in memory, so after a rotation the knots
// of one wave mostly share their sort keys (one counter increment per key and
// wave in the binning) and the scatter writes runs of the sorted order.  The
// spreading sums are exact integers, so the scores do not depend on it.
std::vector<int64_t> morton_order(const corr_ball* balls, int64_t n) {
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = std::numeric_limits<double>::infinity();
        hi[d] = -lo[d];
    }
    for (int64_t i = 0; i < n; ++i) {
        const double x[3] = {balls[i].x, balls[i].y, balls[i].z};
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], x[d]);
            hi[d] = std::max(hi[d], x[d]);
        }
    }
    auto spread = [](uint64_t v) {  // bit b of v to bit 3b
        uint64_t r = 0;
        for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1u) << (3 * b);
        return r;
    };
    std::vector<std::pair<uint64_t, int64_t>> key((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const double x[3] = {balls[i].x, balls[i].y, balls[i].z};
        uint64_t k = 0;
        for (int d = 0; d < 3; ++d) {
            const double t = hi[d] > lo[d] ? (x[d] - lo[d]) / (hi[d] - lo[d]) : 0.0;
            k |= spread((uint64_t)std::min(1023.0, std::max(0.0, std::floor(t * 1024.0)))) << d;
        }
        key[(size_t)i] = {k, i};
    }
    std::sort(key.begin(), key.end());
    std::vector<int64_t> order((size_t)n);
    for (int64_t i = 0; i < n; ++i) order[(size_t)i] = key[(size_t)i].second;
    return order;
}

void upload_shape(corr_ctx* c, DevMem& mem, Shape& s, const corr_ball* balls, double dk) {
    const Expansion& e = s.ex;
    const int64_t n = s.n;
    s.pos = mem.alloc<double>((size_t)3 * std::max<int64_t>(n, 1));
    s.rad = mem.alloc<double>((size_t)std::max<int64_t>(n, 1));
    s.wts = mem.alloc<float>((size_t)e.q * std::max<int64_t>(n, 1));
    s.vtab = mem.alloc<float>((size_t)e.q * c->g.m2n);
    if (n > 0) {
        std::vector<double> pos((size_t)3 * n);
        std::vector<float> w((size_t)e.q * n);
        std::vector<double> lrow(e.p);
        const std::vector<int64_t> order = morton_order(balls, n);
        for (int64_t i = 0; i < n; ++i) {
            const corr_ball& b = balls[order[(size_t)i]];
            pos[3 * i] = b.x;
            pos[3 * i + 1] = b.y;
            pos[3 * i + 2] = b.z;
            lagrange_row(e, std::min(std::max(b.r, e.rlo), e.rhi), lrow.data());
            // equal radii: exact volume ratio (with an offset the two terms scale
            // differently; the lifted kernel is tabulated at the radius itself)
            if (e.p == 1 && e.r0 == 0.0 && !c->lifted) lrow[0] = std::pow(b.r / e.rhi, 3.0);
            for (int q = 0; q < e.q; ++q) {
                double u = 0;
                for (int k = 0; k < e.p; ++k) u += lrow[k] * e.basis[(size_t)k * e.q + q];
                w[(size_t)q * n + i] = (float)(b.w * u);
            }
        }
        upload(s.pos, pos.data(), sizeof(double) * pos.size(), c->stream);
        std::vector<double> rad((size_t)n);
        for (int64_t i = 0; i < n; ++i) rad[i] = balls[order[(size_t)i]].r;
        upload(s.rad, rad.data(), sizeof(double) * rad.size(), c->stream);
        upload(s.wts, w.data(), sizeof(float) * w.size(), c->stream);
        // fixed-point scale: one knot adds w_ic times window values <= 1 to a
        // sum, so with 2^30 / max |w_ic| every addend fits an int32 (converted
        // in one instruction) and a sum of at most 2^31 knots fits int64
        double bound = 0;
        for (int64_t i = 0; i < n; ++i)
            for (int q = 0; q < e.q; ++q) bound = std::max(bound, (double)std::fabs(w[(size_t)q * n + i]));
        int ex2 = 30;
        if (bound > 0) ex2 = (int)std::floor(std::log2(std::ldexp(1.0, 30) / bound));
        ex2 = std::min(ex2, 100);
        if (ex2 < -100) fail(CORR_EUNSUPPORTED, "ball weights too large for the spreading sums");
        s.fix_scale = (float)std::ldexp(1.0, ex2);
    }
    double* d_nodes = mem.alloc<double>(e.p);
    double* d_basis = mem.alloc<double>((size_t)e.p * e.q);
    upload(d_nodes, e.nodes.data(), sizeof(double) * e.p, c->stream);
    upload(d_basis, e.basis.data(), sizeof(double) * e.p * e.q, c->stream);
    s.d_nodes = d_nodes;
    if (!c->lifted)
        hip_check(corr::launch_ball_table(c->g, dk, d_nodes, d_basis, e.p, e.q, e.rref, e.r0, e.lam, s.vtab,
                                          c->stream),
                  "ball table");
}

hipEvent_t take_event(corr_ctx* c) {
    if (!c->spare.empty()) {
        hipEvent_t e = c->spare.back();
        c->spare.pop_back();
        return e;
    }
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    return e;
}

// Launch one stage, bracketed by timing events when profiling is on.
// Failure paths are testable from the host: with the environment variable
// CORR_TEST_FAIL_STAGE set to a stage id, that stage reports a launch failure
// (CORR_EHIP) instead of launching, like CORR_TEST_MAX_BYTES does for device
// allocations.
template <class L>
void stage(corr_ctx* c, int id, const char* what, L&& launch) {
    if (const char* f = std::getenv("CORR_TEST_FAIL_STAGE"))
        if (*f && std::atoi(f) == id) fail(CORR_EHIP, "%s: launch failure forced by CORR_TEST_FAIL_STAGE", what);
    hipEvent_t a = nullptr, b = nullptr;
    if (c->profiling) {
        a = take_event(c);
        b = take_event(c);
        hip_check(hipEventRecord(a, c->stream), "hipEventRecord");
    }
    hip_check(launch(), what);
    if (c->profiling) {
        hip_check(hipEventRecord(b, c->stream), "hipEventRecord");
        c->marks.push_back({id, a, b});
    }
}

corr::Occupancy occupancy(const corr_ctx* c, const Shape& s) {
    corr::Occupancy o;
    o.bin_start = c->ws->bin_start;
    o.tile_live = c->ws->tile_live;
    o.nk = s.n;
    return o;
}

// Stages a0..a3 for S rotations of one shape; quats are device [S][4].
void run_spectrum_stages(corr_ctx* c, const Shape& s, const double* d_quats, int S) {
    const Geom& g = c->g;
    const int q = s.ex.q;
    c->last_S = S;
    c->last_q = q;
    c->last_nk = s.n;
    c->last_ws = c->ws;
    stage(c, CORR_STAGE_ROTATE, "rotate", [&] {
        return corr::launch_rotate_bin(g, d_quats, S, s.pos, s.n, c->ws->rec, c->ws->rank, c->ws->counts,
                                       c->ws->bin_start, c->ws->plan, c->stream);
    });
    stage(c, CORR_STAGE_BIN, "bin", [&] {
        return corr::launch_scatter_plan(g, S, q, occupancy(c, s), c->ws->rec, s.wts, c->ws->rank,
                                         c->ws->scell, c->ws->skbw, c->ws->swts, c->ws->plan, c->ws->list, c->stream);
    });
    stage(c, CORR_STAGE_SPREAD_FFT_X, "spread + fft x", [&] {
        return corr::launch_spread_fftx(g, S, occupancy(c, s), c->ws->plan, c->ws->list, c->ws->scell, c->ws->skbw,
                                        c->ws->swts, q, s.fix_scale, c->ws->buf1, c->twm, c->ws->work, c->stream);
    });
    stage(c, CORR_STAGE_FFT_Y, "fft y", [&] {
        return corr::launch_fft_y(g, S, q, occupancy(c, s), c->ws->buf1, reinterpret_cast<float2*>(c->ws->buf0),
                                  c->twm, c->stream);
    });
}

void stage_quats(corr_ctx* c, const double* q, int S);

// The lifted score's fixed side of the slice at height h into out
// ([q_B][n][n][half]), from A's component spectra (computed first if
// `components`): the node-pair kernel table of that height, then
// H[p'] = sum_p G_A[p] table[p][p'] per mode.
void lifted_fixed_side(corr_ctx* c, double h, float2* out, bool components) {
    const Geom& g = c->g;
    if (components) {
        run_spectrum_stages(c, c->A, c->ident_q, 1);
        stage(c, CORR_STAGE_FFT_Z_SPECTRUM, "fft z components (A)", [&] {
            return corr::launch_fft_z_components(g, reinterpret_cast<float2*>(c->ws->buf0), 1, c->A.ex.q,
                                                 occupancy(c, c->A), c->deconv, c->lift_ga, c->twm, c->stream);
        });
    }
    hip_check(corr::launch_lift_table(g, 2.0 * M_PI / c->box, c->A.d_nodes, c->A.ex.q, c->B.d_nodes, c->B.ex.q, h,
                                      c->lift_tab, c->stream),
              "lifted kernel table");
    hip_check(corr::launch_lift_h(g, c->lift_ga, c->A.ex.q, c->lift_tab, c->B.ex.q, out, c->stream),
              "lifted fixed side");
}

// The fixed shape's spectrum (unturned) into fa.
void fixed_spectrum(corr_ctx* c, const Shape& a, float2* fa) {
    if (c->lifted) {
        lifted_fixed_side(c, 0.0, fa, true);
        return;
    }
    run_spectrum_stages(c, a, c->ident_q, 1);
    stage(c, CORR_STAGE_FFT_Z_SPECTRUM, "fft z (A)", [&] {
        return corr::launch_fft_z_spectrum(c->g, reinterpret_cast<float2*>(c->ws->buf0), 1, a.ex.q,
                                           occupancy(c, a), a.vtab, c->deconv, fa, c->twm, c->stream);
    });
}

corr::WsReq ws_req(const corr_ctx* c);

// Replace the context's own workspace by one of `slots` slots for the current
// plan (ws_req).  The new one is allocated first: if that fails, the old one
// stays in use.  The last pass's occupancy record is dropped with the old one.
void replace_workspace(corr_ctx* c, int slots) {
    hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    auto* nw = new corr::Workspace();
    try {
        nw->allocate(slots, ws_req(c), c->stream);
    } catch (...) {
        nw->release();
        delete nw;
        throw;
    }
    c->gs.drop_graph();
    c->shape_gen++;
    if (c->last_ws == c->ws) {
        c->last_ws = nullptr;
        c->last_S = 0;
    }
    c->ws->release();
    delete c->ws;
    c->ws = nw;
}

// Make the context's stream wait for a pending A spectrum.
void join_a(corr_ctx* c) {
    if (!c->a_pending) return;
    hip_check(hipStreamWaitEvent(c->stream, c->a_done, 0), "hipStreamWaitEvent");
    c->a_pending = false;
}

// A's spectrum into fa.  A context with a workspace of its own computes it on
// a private side stream of default priority, forked from the context's stream
// and with buffers of its own, so that it overlaps the rotated shape's stages
// of the next evaluation; the evaluation joins it before the product, and
// every other call that touches the context's device state joins it first.
void prepare_a(corr_ctx* c) {
    if (!c->own_ws) {
        fixed_spectrum(c, c->A, c->fa);
        return;
    }
    if (!c->side) {
        hip_check(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "hipStreamCreate");
        hip_check(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming), "hipEventCreate");
        hip_check(hipEventCreateWithFlags(&c->a_done, hipEventDisableTiming), "hipEventCreate");
    }
    if (!c->ws_a) {
        auto* w = new corr::Workspace();
        try {
            w->allocate(1, ws_req(c), c->stream);  // its counter clearing is on `stream`, before the fork
        } catch (...) {
            w->release();
            delete w;
            throw;
        }
        c->ws_a = w;
    }
    hip_check(hipEventRecord(c->fork_ev, c->stream), "hipEventRecord");
    hip_check(hipStreamWaitEvent(c->side, c->fork_ev, 0), "hipStreamWaitEvent");
    // on every exit, also after a failed launch: the context's stream and
    // buffers come back, and whatever reached the side stream is joined
    struct Swap {
        corr_ctx* c;
        hipStream_t st;
        corr::Workspace* ws;
        ~Swap() {
            c->stream = st;
            c->ws = ws;
            c->a_pending = hipEventRecord(c->a_done, c->side) == hipSuccess;
            if (!c->a_pending) (void)hipStreamSynchronize(c->side);
        }
    } swap{c, c->stream, c->ws};
    c->stream = c->side;
    c->ws = c->ws_a;
    fixed_spectrum(c, c->A, c->fa);
}

// host quaternions -> pinned staging -> device, S at a time
void stage_quats(corr_ctx* c, const double* q, int S) {
    hip_check(hipEventSynchronize(c->ws->quat_done), "event sync");
    std::memcpy(c->ws->host_quats, q, sizeof(double) * 4 * S);
    hip_check(hipMemcpyAsync(c->ws->quats, c->ws->host_quats, sizeof(double) * 4 * S, hipMemcpyHostToDevice, c->stream), "quat H2D");
    hip_check(hipEventRecord(c->ws->quat_done, c->stream), "event");
}

void validate_quats(const double* q, int64_t n) {
    if (n > 0 && !q) fail(CORR_EINVAL, "NULL quaternion array");
    for (int64_t i = 0; i < n; ++i) {
        double s = 0;
        for (int k = 0; k < 4; ++k) {
            if (!std::isfinite(q[4 * i + k])) fail(CORR_EINVAL, "quaternion %lld has a non-finite entry", (long long)i);
            s += q[4 * i + k] * q[4 * i + k];
        }
        if (std::sqrt(s) < 1e-12) fail(CORR_EINVAL, "quaternion %lld has norm < 1e-12", (long long)i);
    }
}

void destroy_ctx(corr_ctx* c);

// Validate one pair and its grid, plan the window, grids and radius
// expansions, build the tables and upload both shapes (no workspace yet).
corr_ctx* plan_pair(const corr_ball* A, int64_t nA, const corr_ball* B, int64_t nB, const corr_grid* grid,
                    void* hip_stream, const char* who) {
    if (!grid) fail(CORR_EINVAL, "%sgrid is NULL", who);
    validate_balls(A, nA, "A");
    validate_balls(B, nB, "B");
    const corr_grid& gr = *grid;
    if (gr.n != 16 && gr.n != 32 && gr.n != 64 && gr.n != 128 && gr.n != 256)
        fail(CORR_EUNSUPPORTED, "%sgrid n = %d; supported: 16, 32, 64, 128, 256", who, gr.n);
    if (!std::isfinite(gr.box) || !(gr.box > 0)) fail(CORR_EINVAL, "%sgrid box must be finite and > 0", who);
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(gr.origin[d])) fail(CORR_EINVAL, "%sgrid origin must be finite", who);
    const double sigma = gr.sigma == 0 ? 2.0 : gr.sigma;
    if (sigma != 2.0) fail(CORR_EUNSUPPORTED, "%ssigma = %g; supported: 2", who, sigma);
    const int w = gr.kb_width == 0 ? 8 : gr.kb_width;
    // at w = 4 the window alone leaves a relative error of ~1e-3 (sigma = 2),
    // above the 1e-4 tolerance of the path; 6 leaves ~1e-5, 8 ~1e-7
    if (w < 6 || w > 12 || (w & 1))
        fail(CORR_EUNSUPPORTED, "%skb_width = %d; supported: even 6..12 (narrower windows miss the 1e-4 tolerance)",
             who, w);
    const double tol = gr.tol == 0 ? 1e-6 : gr.tol;
    if (!std::isfinite(tol) || !(tol > 0) || tol >= 1) fail(CORR_EINVAL, "%stol must be in (0, 1)", who);
    if (gr.flags & ~(CORR_DETERMINISTIC | CORR_SC_SCORE | CORR_LIFTED_SCORE))
        fail(CORR_EINVAL, "%sunknown flag bits 0x%x", who, gr.flags);
    if ((gr.flags & CORR_LIFTED_SCORE) && (gr.flags & CORR_SC_SCORE))
        fail(CORR_EINVAL, "%sCORR_LIFTED_SCORE and CORR_SC_SCORE exclude each other", who);
    if (gr.flags & CORR_LIFTED_SCORE) {
        if (!std::isfinite(gr.lift_range) || gr.lift_range < 0) fail(CORR_EINVAL, "%slift_range must be finite and >= 0", who);
    } else if (gr.lift_range != 0) {
        fail(CORR_EINVAL, "%slift_range needs CORR_LIFTED_SCORE", who);
    }
    if (gr.flags & CORR_SC_SCORE) {
        if (!std::isfinite(gr.sc_offset) || gr.sc_offset < 0) fail(CORR_EINVAL, "%ssc_offset must be finite and >= 0", who);
        if (!std::isfinite(gr.sc_lambda) || gr.sc_lambda < 0) fail(CORR_EINVAL, "%ssc_lambda must be finite and >= 0", who);
    } else if (gr.sc_offset != 0 || gr.sc_lambda != 0) {
        fail(CORR_EINVAL, "%ssc_offset and sc_lambda need CORR_SC_SCORE", who);
    }
    if (gr.batch < 0 || gr.batch > 256) fail(CORR_EINVAL, "%sbatch = %d; allowed 0..256", who, gr.batch);

    corr_ctx* c = new corr_ctx();
    try {
        hip_check(hipGetDevice(&c->device), "hipGetDevice");
        c->stream = static_cast<hipStream_t>(hip_stream);
        c->box = gr.box;
        std::memcpy(c->origin, gr.origin, sizeof c->origin);
        c->sigma = sigma;
        c->tol = tol;
        c->flags = gr.flags;
        c->sc_r0 = (gr.flags & CORR_SC_SCORE) ? gr.sc_offset : 0.0;
        c->sc_lam = (gr.flags & CORR_SC_SCORE) ? gr.sc_lambda : 0.0;
        Geom& g = c->g;
        g.n = gr.n;
        g.m = (int)std::lround(sigma * gr.n);
        g.w = w;
        g.half = gr.n / 2;
        g.m2n = 3 * (g.half - 1) * (g.half - 1) + 1;
        // window shape for oversampling sigma (Beatty, Nishimura & Pauly, 2005)
        const double beta = M_PI * std::sqrt((w / sigma) * (w / sigma) * (sigma - 0.5) * (sigma - 0.5) - 0.8);
        g.beta = (float)beta;
        g.inv_i0beta = (float)(1.0 / std::cyl_bessel_i(0.0, (double)g.beta));
        g.inv_hf = g.m / gr.box;
        int cus = 0;
        hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device), "CU count");
        g.spread_wgs = 2 * std::max(cus, 1);
        const double dk = 2.0 * M_PI / gr.box;
        if (gr.flags & CORR_LIFTED_SCORE) {
            // heights within the planned range that leave every pair's cones
            // meeting (r_i + rho_j - h >= half the smallest radius sum)
            double alo, ahi, blo, bhi;
            radius_range(A, nA, alo, ahi);
            radius_range(B, nB, blo, bhi);
            c->lifted = true;
            c->lift_lo = -gr.lift_range;
            c->lift_hi = std::min(gr.lift_range, 0.5 * (alo + blo));
        }

        setup_shape(c, c->A, A, nA, dk, B, nB);
        setup_shape(c, c->B, B, nB, dk, A, nA);
        c->qmax = std::max(c->A.ex.q, c->B.ex.q);
        c->nkmax = std::max<int64_t>(std::max(nA, nB), 1);

        hipDeviceProp_t prop;
        hip_check(hipGetDeviceProperties(&prop, c->device), "hipGetDeviceProperties");
        const size_t need = corr::max_lds_bytes(g, c->qmax);  // largest dynamic LDS of any stage
        if (need > prop.sharedMemPerBlock)
            fail(CORR_EUNSUPPORTED, "%sgrid n = %d needs %zu bytes of LDS per workgroup; device has %zu", who, g.n,
                 need, (size_t)prop.sharedMemPerBlock);

        std::vector<float2> tw(g.m);
        for (int j = 0; j < g.m; ++j)
            tw[j] = make_float2((float)std::cos(2 * M_PI * j / g.m), (float)-std::sin(2 * M_PI * j / g.m));
        c->twm = c->mem.alloc<float2>(g.m);
        upload(c->twm, tw.data(), sizeof(float2) * g.m, c->stream);
        tw.resize(g.n);
        for (int j = 0; j < g.n; ++j)
            tw[j] = make_float2((float)std::cos(2 * M_PI * j / g.n), (float)-std::sin(2 * M_PI * j / g.n));
        c->twn = c->mem.alloc<float2>(g.n);
        upload(c->twn, tw.data(), sizeof(float2) * g.n, c->stream);
        c->deconv = c->mem.alloc<double>(g.n);
        c->phase = c->mem.alloc<double2>((size_t)3 * g.n);
        hip_check(corr::launch_deconv_tables(g, c->box, c->origin, c->deconv, c->phase, c->stream), "deconv tables");
        upload_shape(c, c->mem, c->A, A, dk);
        upload_shape(c, c->mem, c->B, B, dk);
        c->host_a.assign(A, A + nA);
        // the fixed side of a slice: F_A, or for the lifted score one table
        // per component of B
        c->fa = c->mem.alloc<float2>((size_t)(c->lifted ? c->B.ex.q : 1) * g.n * g.n * g.half);
        if (c->lifted) {
            c->lift_tab = c->mem.alloc<float>((size_t)c->A.ex.q * c->B.ex.q * g.m2n);
            c->lift_ga = c->mem.alloc<float2>((size_t)c->A.ex.q * g.n * g.n * g.half);
        }
        static const double ident[4] = {1, 0, 0, 0};
        c->ident_q = c->mem.alloc<double>(4);
        upload(c->ident_q, ident, sizeof ident, c->stream);
    } catch (...) {
        destroy_ctx(c);
        throw;
    }
    return c;
}

corr::WsReq ws_req(const corr_ctx* c) {
    corr::WsReq r;
    const Geom& g = c->g;
    r.buf0 = (size_t)2 * c->qmax * g.m * g.n * g.half;
    r.buf1 = (size_t)c->qmax * g.m * g.m * g.half;
    r.nk = (size_t)c->nkmax;
    r.nkw = (size_t)c->nkmax * 3 * g.w;
    r.nkq = (size_t)c->nkmax * c->qmax;
    r.counts = (size_t)corr::bin_keys_max(g.m);
    r.bins = (size_t)corr::bin_keys_max(g.m) + 1;
    r.blocks = (size_t)corr::ifft_x_blocks_max(g);  // any inverse-x width
    r.tiles = (size_t)g.m * corr::spread_tiles_max(g);
    r.list = (size_t)corr::plan_buckets() * r.tiles;
    return r;
}

// Outputs of one evaluation; slice k's arrays follow slice k-1's (n_rot rotations each).
struct EvalOut {
    float* scores = nullptr;
    float* peak_val = nullptr;
    int64_t* peak_idx = nullptr;
    unsigned* mask = nullptr;
    int64_t* count = nullptr;
    float thr = 0.f;
};

void check_eval_args(int64_t n_rot, const EvalOut& o);

// Score n_rot rotations of B (validated here) against each fixed spectrum in
// fas, batch by batch: B is spread and transformed once per batch, then each
// slice takes the product and inverse passes (the inverse y pass works in
// place, so B's transformed components stay for the next slice).
void eval_impl(corr_ctx* c, const double* quat_wxyz, int64_t n_rot, const std::vector<const float2*>& fas,
               const EvalOut& o, const double* d_quats = nullptr) {
    check_eval_args(n_rot, o);
    if (!d_quats) validate_quats(quat_wxyz, n_rot);
    const Geom& g = c->g;
    const size_t n3 = (size_t)g.n * g.n * g.n;
    const int nb = corr::ifft_x_blocks(g);
    const int slots = c->slots_eff > 0 ? c->slots_eff : c->ws->slots;
    for (int64_t r0 = 0; r0 < n_rot; r0 += slots) {
        const int S = (int)std::min<int64_t>(slots, n_rot - r0);
        // rotations already on the device (graph replay), or staged per batch
        if (!d_quats) stage_quats(c, quat_wxyz + 4 * r0, S);
        run_spectrum_stages(c, c->B, d_quats ? d_quats + 4 * r0 : c->ws->quats, S);
        if (c->lifted) {
            // B's component z transforms once (into buf1, free after the y
            // pass), then per slice: sum_p' H[p'] conj(G_B[p']), inverse z into
            // buf0 (free after the z pass), inverse y in place, inverse x
            float2* comps = c->ws->buf1;
            float2* prod = reinterpret_cast<float2*>(c->ws->buf0);
            stage(c, CORR_STAGE_FFT_Z_SPECTRUM, "fft z components (B)", [&] {
                return corr::launch_fft_z_components(g, prod, S, c->B.ex.q, occupancy(c, c->B), nullptr, comps,
                                                     c->twm, c->stream);
            });
            join_a(c);
            for (size_t k = 0; k < fas.size(); ++k) {
                const size_t first = (size_t)k * n_rot + r0;
                stage(c, CORR_STAGE_FFT_Z_PRODUCT, "lifted product", [&] {
                    return corr::launch_lift_product_ifft_z(g, comps, S, c->B.ex.q, c->phase, fas[k], prod, c->twn,
                                                            c->stream);
                });
                stage(c, CORR_STAGE_IFFT_Y, "ifft y",
                      [&] { return corr::launch_ifft_y(g, prod, S, prod, c->twn, c->stream); });
                stage(c, CORR_STAGE_IFFT_X, "ifft x", [&] {
                    return corr::launch_ifft_x(g, prod, S, o.scores ? o.scores + first * n3 : nullptr,
                                               o.mask ? o.mask + first * (n3 / 32) : nullptr, o.thr, c->ws->pval,
                                               c->ws->pidx, o.count ? c->ws->pcnt : nullptr, c->twn, c->stream);
                });
                if (o.peak_val || o.count)
                    stage(c, CORR_STAGE_PEAK, "peak", [&] {
                        return corr::launch_peak_final(c->ws->pval, c->ws->pidx, c->ws->pcnt, S, nb,
                                                       o.peak_val ? o.peak_val + first : nullptr,
                                                       o.peak_idx ? o.peak_idx + first : nullptr,
                                                       o.count ? o.count + first : nullptr, c->stream);
                    });
            }
            continue;
        }
        // several slices: B's z sums once, into the second half of buf1
        // (buf1 holds q m^2 n/2 >= 2 n^2 n/2 values per slot)
        float2* zsums = c->ws->buf1 + (size_t)c->ws->slots * g.n * g.n * g.half;
        if (fas.size() > 1)
            stage(c, CORR_STAGE_FFT_Z_SPECTRUM, "fft z sums (B)", [&] {
                return corr::launch_fft_z_spectrum(g, reinterpret_cast<float2*>(c->ws->buf0), S, c->B.ex.q,
                                                   occupancy(c, c->B), c->B.vtab, nullptr, zsums, c->twm, c->stream);
            });
        join_a(c);  // F_A is read from here on
        for (size_t k = 0; k < fas.size(); ++k) {
            const size_t first = (size_t)k * n_rot + r0;  // this slice's first rotation of the batch
            stage(c, CORR_STAGE_FFT_Z_PRODUCT, "fft z product", [&] {
                if (fas.size() > 1)
                    return corr::launch_product_ifft_z(g, zsums, S, c->phase, fas[k], c->ws->buf1, c->twn, c->stream);
                return corr::launch_fft_z_product(g, reinterpret_cast<float2*>(c->ws->buf0), S, c->B.ex.q,
                                                  occupancy(c, c->B), c->B.vtab, c->phase, fas[k], c->ws->buf1,
                                                  c->twm, c->twn, c->stream);
            });
            stage(c, CORR_STAGE_IFFT_Y, "ifft y", [&] {
                return corr::launch_ifft_y(g, c->ws->buf1, S, c->ws->buf1, c->twn, c->stream);
            });
            stage(c, CORR_STAGE_IFFT_X, "ifft x", [&] {
                return corr::launch_ifft_x(g, c->ws->buf1, S, o.scores ? o.scores + first * n3 : nullptr,
                                           o.mask ? o.mask + first * (n3 / 32) : nullptr, o.thr, c->ws->pval,
                                           c->ws->pidx, o.count ? c->ws->pcnt : nullptr, c->twn, c->stream);
            });
            if (o.peak_val || o.count)
                stage(c, CORR_STAGE_PEAK, "peak", [&] {
                    return corr::launch_peak_final(c->ws->pval, c->ws->pidx, c->ws->pcnt, S, nb,
                                                   o.peak_val ? o.peak_val + first : nullptr,
                                                   o.peak_idx ? o.peak_idx + first : nullptr,
                                                   o.count ? o.count + first : nullptr, c->stream);
                });
        }
    }
}

// ---- graph replay ------------------------------------------------------------

// Copy n host rotations into gs's device array (grown on demand, which drops
// the captured graph: it reads the old array) on stream st.
const double* graph_quats(GraphState& gs, hipStream_t st, const double* q, int64_t n) {
    if (n > gs.cap_rot) {
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        gs.drop_graph();
        if (gs.d_quats) (void)hipFree(gs.d_quats);
        if (gs.h_quats) (void)hipHostFree(gs.h_quats);
        gs.d_quats = nullptr;
        gs.h_quats = nullptr;
        gs.cap_rot = 0;
        const int64_t cap = std::max<int64_t>(n, 64);
        hip_check(hipMalloc((void**)&gs.d_quats, sizeof(double) * 4 * cap), "hipMalloc (graph rotations)");
        hip_check(hipHostMalloc((void**)&gs.h_quats, sizeof(double) * 4 * cap, hipHostMallocDefault), "hipHostMalloc");
        gs.cap_rot = cap;
        if (!gs.copied) hip_check(hipEventCreateWithFlags(&gs.copied, hipEventDisableTiming), "hipEventCreate");
    } else {
        hip_check(hipEventSynchronize(gs.copied), "event sync");  // h_quats free again
    }
    std::memcpy(gs.h_quats, q, sizeof(double) * 4 * n);
    hip_check(hipMemcpyAsync(gs.d_quats, gs.h_quats, sizeof(double) * 4 * n, hipMemcpyHostToDevice, st),
              "rotations H2D");
    hip_check(hipEventRecord(gs.copied, st), "hipEventRecord");
    return gs.d_quats;
}

// While capturing: the contexts' launches go to the capture stream, without
// per-stage timing events.
struct CaptureScope {
    std::vector<corr_ctx*> cs;
    std::vector<hipStream_t> streams;
    std::vector<bool> prof;
    CaptureScope(const std::vector<corr_ctx*>& ctxs, hipStream_t cap) : cs(ctxs) {
        for (corr_ctx* c : cs) {
            streams.push_back(c->stream);
            prof.push_back(c->profiling);
            c->stream = cap;
            c->profiling = false;
        }
    }
    ~CaptureScope() {
        for (size_t i = 0; i < cs.size(); ++i) {
            cs[i]->stream = streams[i];
            cs[i]->profiling = prof[i];
        }
    }
};

// Launch the graph captured for `key` on st, capturing it first (body(stream)
// enqueues the evaluation) if there is none or it was captured for another key.
template <class Body>
void graph_launch(GraphState& gs, hipStream_t st, std::vector<uint64_t> key, const std::vector<corr_ctx*>& ctxs,
                  corr_ctx* timed, Body&& body) {
    key.push_back((uint64_t)(uintptr_t)gs.d_quats);
    if (!gs.exec || key != gs.key) {
        gs.drop_graph();
        if (!gs.cap) hip_check(hipStreamCreateWithFlags(&gs.cap, hipStreamNonBlocking), "hipStreamCreate");
        hip_check(hipStreamBeginCapture(gs.cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        try {
            CaptureScope scope(ctxs, gs.cap);
            body();
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(gs.cap, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        hip_check(hipStreamEndCapture(gs.cap, &gs.graph), "hipStreamEndCapture");
        hip_check(hipGraphInstantiate(&gs.exec, gs.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        gs.key = std::move(key);
    }
    if (timed)
        stage(timed, CORR_STAGE_GRAPH, "hipGraphLaunch", [&] { return hipGraphLaunch(gs.exec, st); });
    else
        hip_check(hipGraphLaunch(gs.exec, st), "hipGraphLaunch");
}

void check_eval_args(int64_t n_rot, const EvalOut& o) {
    if (n_rot < 0) fail(CORR_EINVAL, "n_rot < 0");
    if ((o.peak_val == nullptr) != (o.peak_idx == nullptr))
        fail(CORR_EINVAL, "peak_val and peak_idx must both be set or both be NULL");
    if (!std::isfinite(o.thr)) fail(CORR_EINVAL, "threshold must be finite");
}

// An evaluation: enqueued launch by launch, or (graph mode) as one graph launch.
void eval_entry(corr_ctx* c, const double* quat_wxyz, int64_t n_rot, const std::vector<const float2*>& fas,
                const EvalOut& o) {
    if (!c->graph) {
        eval_impl(c, quat_wxyz, n_rot, fas, o);
        return;
    }
    check_eval_args(n_rot, o);
    validate_quats(quat_wxyz, n_rot);
    if (n_rot == 0) return;
    join_a(c);  // outside the capture: the graph waits on nothing it did not record
    const double* dq = graph_quats(c->gs, c->stream, quat_wxyz, n_rot);
    float thr_bits = o.thr;
    uint32_t tb;
    std::memcpy(&tb, &thr_bits, 4);
    std::vector<uint64_t> key = {1, c->shape_gen, (uint64_t)n_rot, (uint64_t)(uintptr_t)o.scores,
                                 (uint64_t)(uintptr_t)o.peak_val, (uint64_t)(uintptr_t)o.peak_idx,
                                 (uint64_t)(uintptr_t)o.mask, (uint64_t)(uintptr_t)o.count, tb};
    for (const float2* f : fas) key.push_back((uint64_t)(uintptr_t)f);
    graph_launch(c->gs, c->stream, std::move(key), {c}, c, [&] { eval_impl(c, nullptr, n_rot, fas, o, dq); });
}

void eval_plain(corr_ctx* c, const double* quat_wxyz, int64_t n_rot, float* scores_dev, float* peak_val_dev,
                int64_t* peak_idx_dev) {
    EvalOut o;
    o.scores = scores_dev;
    o.peak_val = peak_val_dev;
    o.peak_idx = peak_idx_dev;
    eval_entry(c, quat_wxyz, n_rot, {c->fa}, o);
}

// Plan and compute the offset slices of A (corr_set_offsets).
void set_offsets(corr_ctx* c, const double* offsets, int32_t n) {
    join_a(c);
    if (c->flags & CORR_SC_SCORE)
        fail(CORR_EUNSUPPORTED, "offset slices with CORR_SC_SCORE: its kernel already offsets the balls");
    if (n < 0 || n > CORR_MAX_SLICES) fail(CORR_EINVAL, "n_offsets = %d; allowed 0..%d", n, CORR_MAX_SLICES);
    if (n > 0 && !offsets) fail(CORR_EINVAL, "NULL offsets with n_offsets = %d", n);
    if (c->lifted) {
        // slice heights of the lifted correlation: each slice's fixed side from
        // A's component spectra (kept since corr_create / corr_prepare_a)
        for (int k = 0; k < n; ++k)
            if (!std::isfinite(offsets[k]) || offsets[k] < c->lift_lo || offsets[k] > c->lift_hi)
                fail(CORR_EINVAL, "height %d (%g) is outside the planned range [%g, %g] (corr_grid.lift_range)", k,
                     offsets[k], c->lift_lo, c->lift_hi);
        std::vector<Slice> ns(n);
        DevMem nm;
        try {
            for (int k = 0; k < n; ++k) {
                ns[k].delta = offsets[k];
                ns[k].fa = nm.alloc<float2>((size_t)c->B.ex.q * c->g.n * c->g.n * c->g.half);
                lifted_fixed_side(c, offsets[k], ns[k].fa, false);
            }
            hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
        } catch (...) {
            (void)hipStreamSynchronize(c->stream);
            nm.release();
            throw;
        }
        c->slice_mem.release();
        c->slices = std::move(ns);
        c->slice_mem = nm;
        c->shape_gen++;
        return;
    }
    double rmin = HUGE_VAL;
    for (const corr_ball& b : c->host_a) rmin = std::min(rmin, b.r);
    for (int k = 0; k < n; ++k) {
        if (!std::isfinite(offsets[k])) fail(CORR_EINVAL, "offset %d is not finite", k);
        if (!c->host_a.empty() && !(rmin + offsets[k] > 0))
            fail(CORR_EINVAL, "offset %d (%g) leaves a ball of A with radius <= 0 (smallest radius %g)", k, offsets[k],
                 rmin);
    }
    const double dk = 2.0 * M_PI / c->box;
    const int64_t na = (int64_t)c->host_a.size();
    std::vector<Slice> ns(n);
    DevMem nm;
    try {
        std::vector<corr_ball> grown(c->host_a);
        int qmax = c->qmax;
        for (int k = 0; k < n; ++k) {
            for (int64_t i = 0; i < na; ++i) grown[i].r = c->host_a[i].r + offsets[k];
            ns[k].delta = offsets[k];
            setup_shape(c, ns[k].A, grown.data(), na, dk);
            qmax = std::max(qmax, ns[k].A.ex.q);
            upload_shape(c, nm, ns[k].A, grown.data(), dk);
            ns[k].fa = nm.alloc<float2>((size_t)c->g.n * c->g.n * c->g.half);
        }
        if (qmax > c->qmax) {  // a slice needs more components than the workspace holds
            if (!c->own_ws) fail(CORR_EUNSUPPORTED, "offset slices need a larger shared workspace");
            hipDeviceProp_t prop;
            hip_check(hipGetDeviceProperties(&prop, c->device), "hipGetDeviceProperties");
            if (corr::max_lds_bytes(c->g, qmax) > prop.sharedMemPerBlock)
                fail(CORR_EUNSUPPORTED, "offset slices need %d radius components: too much LDS", qmax);
            const int old_q = c->qmax;
            c->qmax = qmax;  // ws_req plans for the slices' components
            try {
                replace_workspace(c, c->ws->slots);
            } catch (...) {
                c->qmax = old_q;
                throw;
            }
        }
        for (int k = 0; k < n; ++k) fixed_spectrum(c, ns[k].A, ns[k].fa);
        hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    } catch (...) {
        (void)hipStreamSynchronize(c->stream);
        nm.release();
        throw;
    }
    hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    c->slice_mem.release();
    c->slices = std::move(ns);
    c->slice_mem = nm;
    c->shape_gen++;
}

template <class F>
int guarded(corr_ctx* c, F&& body) {
    try {
        body();
        return CORR_OK;
    } catch (const CorrError& e) {
        if (c) c->err = e.msg;
        else g_thread_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        if (c) c->err = "host allocation failed";
        else g_thread_error = "host allocation failed";
        return CORR_ENOMEM;
    } catch (...) {
        if (c) c->err = "unexpected internal error";
        else g_thread_error = "unexpected internal error";
        return CORR_EHIP;
    }
}

void destroy_ctx(corr_ctx* c) {
    if (!c) return;
    if (c->side) (void)hipStreamSynchronize(c->side);
    (void)hipStreamSynchronize(c->stream);
    for (auto* g : {&c->q_modes, &c->q_part, &c->q_P, &c->q_t, &c->q_quat, &c->q_tpart})
        if (g->p) (void)hipFree(g->p);
    if (c->q_host) (void)hipHostFree(c->q_host);
    if (c->q_done) (void)hipEventDestroy(c->q_done);
    c->gs.release();
    c->mem.release();
    c->slice_mem.release();
    if (c->own_ws && c->ws) {
        c->ws->release();
        delete c->ws;
    }
    c->ws = nullptr;
    if (c->ws_a) {
        c->ws_a->release();
        delete c->ws_a;
    }
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    if (c->a_done) (void)hipEventDestroy(c->a_done);
    if (c->side) (void)hipStreamDestroy(c->side);
    for (auto& mk : c->marks) {
        (void)hipEventDestroy(mk.a);
        (void)hipEventDestroy(mk.b);
    }
    for (hipEvent_t e : c->spare) (void)hipEventDestroy(e);
    delete c;
}

// ---- launch shapes and the autotuner ---------------------------------------

int cu_count(const corr_ctx* c) {
    int cus = 0;
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device), "CU count");
    return std::max(cus, 1);
}

corr_tuning get_tuning(const corr_ctx* c) {
    corr_tuning t;
    std::memset(&t, 0, sizeof t);
    int def[3];
    t.slots = c->ws->slots;
    t.spread_wgs = c->g.spread_wgs;
    t.cols_y = c->g.cols_y ? c->g.cols_y : (corr::col_choices(c->g.m, 0, def), def[0]);
    t.cols_z = c->g.cols_z ? c->g.cols_z : (corr::col_choices(c->g.m, 1, def), def[0]);
    t.cols_iy = c->g.cols_iy ? c->g.cols_iy : (corr::col_choices(c->g.m, 2, def), def[0]);
    t.pairs_ix = c->g.pairs_ix ? c->g.pairs_ix : (corr::col_choices(c->g.m, 3, def), def[0]);
    t.graph = c->graph ? 1 : 0;
    t.bin_group = corr::bin_group(c->g);
    {
        int tr[2];
        corr::tile_choices(c->g.m, tr);
        t.tile_rows = c->g.tile_rows ? c->g.tile_rows : tr[0];
    }
    return t;
}

// Validate t against the context's choices; then apply it (the workspace is
// reallocated, after the stream has drained, when the slot count changes).
void set_tuning(corr_ctx* c, const corr_tuning& t) {
    join_a(c);
    const int widths[4] = {t.cols_y, t.cols_z, t.cols_iy, t.pairs_ix};
    static const char* names[4] = {"cols_y", "cols_z", "cols_iy", "pairs_ix"};
    for (int p = 0; p < 4; ++p) {
        int ch[3];
        const int k = corr::col_choices(c->g.m, p, ch);
        bool ok = false;
        for (int i = 0; i < k; ++i) ok = ok || ch[i] == widths[p];
        if (!ok) fail(CORR_EINVAL, "%s = %d is not one of this grid's widths (corr_tuning_choices)", names[p], widths[p]);
    }
    const int cus = cu_count(c);
    if (t.spread_wgs < 1 || t.spread_wgs > 2 * cus)
        fail(CORR_EINVAL, "spread_wgs = %d; allowed 1..%d (two per CU)", t.spread_wgs, 2 * cus);
    if (t.slots < 1 || t.slots > 256) fail(CORR_EINVAL, "slots = %d; allowed 1..256", t.slots);
    if (t.graph != 0 && t.graph != 1) fail(CORR_EINVAL, "graph must be 0 or 1");
    {
        int bg[3];
        const int k = corr::bin_choices(c->g.m, bg);
        bool ok = false;
        for (int i = 0; i < k; ++i) ok = ok || bg[i] == t.bin_group;
        if (!ok) fail(CORR_EINVAL, "bin_group = %d is not one of this grid's groups (corr_tuning_choices)", t.bin_group);
        int tr[2];
        const int kt = corr::tile_choices(c->g.m, tr);
        ok = false;
        for (int i = 0; i < kt; ++i) ok = ok || tr[i] == t.tile_rows;
        if (!ok) fail(CORR_EINVAL, "tile_rows = %d is not one of this grid's tile heights (corr_tuning_choices)",
                      t.tile_rows);
    }
    if (t.slots != c->ws->slots) {
        if (!c->own_ws) fail(CORR_EUNSUPPORTED, "the pairs of a batch share their workspace: slots are fixed");
        replace_workspace(c, t.slots);
    }
    Geom& g = c->g;
    if (g.cols_y != t.cols_y || g.cols_z != t.cols_z || g.cols_iy != t.cols_iy || g.pairs_ix != t.pairs_ix ||
        g.spread_wgs != t.spread_wgs || corr::bin_group(g) != t.bin_group || get_tuning(c).tile_rows != t.tile_rows)
        c->shape_gen++;
    g.bin_group = t.bin_group;
    g.tile_rows = t.tile_rows;
    g.cols_y = t.cols_y;
    g.cols_z = t.cols_z;
    g.cols_iy = t.cols_iy;
    g.pairs_ix = t.pairs_ix;
    g.spread_wgs = t.spread_wgs;
    c->graph = t.graph != 0;
}

// Coordinate descent over the launch shapes: each setting in turn takes the
// candidate whose evaluation of these rotations is fastest (the least of
// `reps` timed runs after one untimed run), the others held.  Results do not
// depend on the launch shape, so only time is compared.
corr_tuning autotune(corr_ctx* c, const double* q, int64_t n_rot, float* scores, float* pv, int64_t* pi,
                     int reps, uint32_t flags) {
    if (n_rot < 1) fail(CORR_EINVAL, "autotuning needs n_rot >= 1");
    if (reps < 1 || reps > 100) fail(CORR_EINVAL, "reps = %d; allowed 1..100", reps);
    if (flags & ~CORR_TUNE_WITH_A) fail(CORR_EINVAL, "unknown autotune flag bits 0x%x", flags);
    const bool with_a = (flags & CORR_TUNE_WITH_A) != 0;
    if ((pv == nullptr) != (pi == nullptr)) fail(CORR_EINVAL, "peak_val and peak_idx must both be set or both be NULL");
    validate_quats(q, n_rot);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    const bool prof = c->profiling;
    c->profiling = false;
    const corr_tuning start = get_tuning(c);
    try {
        // the timed unit: corr_eval, or corr_prepare_a + corr_eval (A's spectrum
        // forks off the context's stream after e0 and is joined before e1)
        auto unit = [&] {
            if (with_a) prepare_a(c);
            eval_plain(c, q, n_rot, scores, pv, pi);
        };
        auto timed = [&](const corr_tuning& t) {
            set_tuning(c, t);
            unit();  // untimed: first touch, graph capture
            float best = INFINITY;
            for (int r = 0; r < reps; ++r) {
                hip_check(hipEventRecord(e0, c->stream), "hipEventRecord");
                unit();
                hip_check(hipEventRecord(e1, c->stream), "hipEventRecord");
                hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
                float ms = 0;
                hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                best = std::min(best, ms);
            }
            return best;
        };
        corr_tuning cur = start;
        float cur_ms = timed(cur);
        auto try_field = [&](int32_t corr_tuning::*field, const std::vector<int>& cands) {
            for (int v : cands) {
                if (v == cur.*field) continue;
                corr_tuning t = cur;
                t.*field = v;
                const float ms = timed(t);
                if (ms < cur_ms) {
                    cur = t;
                    cur_ms = ms;
                }
            }
        };
        if (c->own_ws) {
            // rotations per pass: powers of two up to the rotations given,
            // with the workspace under 8 GiB
            const size_t per = ws_req(c).slot_bytes();
            std::vector<int> sl;
            for (int sv = 1; sv <= 256; sv *= 2)
                if ((sv <= n_rot || sv / 2 < n_rot) && (size_t)sv * per <= ((size_t)8 << 30)) sl.push_back(sv);
            try_field(&corr_tuning::slots, sl);
        }
        const int cus = cu_count(c);
        try_field(&corr_tuning::spread_wgs, {cus, cus + cus / 2, 2 * cus});
        int32_t corr_tuning::*fields[4] = {&corr_tuning::cols_y, &corr_tuning::cols_z, &corr_tuning::cols_iy,
                                           &corr_tuning::pairs_ix};
        for (int p = 0; p < 4; ++p) {
            int ch[3];
            const int k = corr::col_choices(c->g.m, p, ch);
            try_field(fields[p], std::vector<int>(ch, ch + k));
        }
        int bg[3];
        const int kb = corr::bin_choices(c->g.m, bg);
        try_field(&corr_tuning::bin_group, std::vector<int>(bg, bg + kb));
        int tr[2];
        const int kt = corr::tile_choices(c->g.m, tr);
        try_field(&corr_tuning::tile_rows, std::vector<int>(tr, tr + kt));
        set_tuning(c, cur);
    } catch (...) {
        (void)hipStreamSynchronize(c->stream);
        try {
            set_tuning(c, start);
        } catch (...) {
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        c->profiling = prof;
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->profiling = prof;
    return get_tuning(c);
}

}  // namespace

extern "C" {

int corr_get_tuning(const corr_ctx* c, corr_tuning* out) {
    if (!c || !out) {
        g_thread_error = "corr_get_tuning: NULL argument";
        return CORR_EINVAL;
    }
    return guarded(const_cast<corr_ctx*>(c), [&] { *out = get_tuning(c); });
}

int corr_set_tuning(corr_ctx* c, const corr_tuning* t) {
    if (!c) {
        g_thread_error = "corr_set_tuning: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] {
        if (!t) fail(CORR_EINVAL, "tuning is NULL");
        set_tuning(c, *t);
    });
}

int corr_tuning_choices(const corr_ctx* c, int32_t pass, int32_t* out3, int32_t* count) {
    if (!c || !out3 || !count) {
        g_thread_error = "corr_tuning_choices: NULL argument";
        return CORR_EINVAL;
    }
    int ch[3];
    const int k = (pass >= 0 && pass < 4) ? corr::col_choices(c->g.m, pass, ch)
                  : pass == 4             ? corr::bin_choices(c->g.m, ch)
                  : pass == 5             ? corr::tile_choices(c->g.m, ch)
                                          : 0;
    if (k == 0) {
        g_thread_error = "corr_tuning_choices: pass must be 0..5";
        return CORR_EINVAL;
    }
    for (int i = 0; i < k; ++i) out3[i] = ch[i];
    *count = k;
    return CORR_OK;
}

int corr_autotune(corr_ctx* c, const double* quat_wxyz, int64_t n_rot, float* scores_dev, float* peak_val_dev,
                  int64_t* peak_idx_dev, int32_t reps, uint32_t flags, corr_tuning* out) {
    if (!c) {
        g_thread_error = "corr_autotune: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] {
        const corr_tuning t = autotune(c, quat_wxyz, n_rot, scores_dev, peak_val_dev, peak_idx_dev, reps, flags);
        if (out) *out = t;
    });
}

int corr_create(const corr_ball* A, int64_t nA, const corr_ball* B, int64_t nB, const corr_grid* grid,
                void* hip_stream, corr_ctx** out) {
    corr_ctx* c = nullptr;
    int rc = guarded(nullptr, [&] {
        if (!out) fail(CORR_EINVAL, "out is NULL");
        *out = nullptr;
        c = plan_pair(A, nA, B, nB, grid, hip_stream, "");
        const corr::WsReq r = ws_req(c);
        int slots = grid->batch;
        if (slots == 0) slots = (int)std::max<size_t>(1, std::min<size_t>(64, ((size_t)4 << 30) / r.slot_bytes()));
        c->ws = new corr::Workspace();
        c->own_ws = true;
        c->ws->allocate(slots, r, c->stream);
        prepare_a(c);
        *out = c;
    });
    if (rc != CORR_OK && c) destroy_ctx(c);
    return rc;
}

int corr_prepare_a(corr_ctx* c) {
    if (!c) {
        g_thread_error = "corr_prepare_a: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] { prepare_a(c); });
}

int corr_eval(corr_ctx* c, const double* quat_wxyz, int64_t n_rot, float* scores_dev, float* peak_val_dev,
              int64_t* peak_idx_dev) {
    if (!c) {
        g_thread_error = "corr_eval: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] { eval_plain(c, quat_wxyz, n_rot, scores_dev, peak_val_dev, peak_idx_dev); });
}

int corr_set_offsets(corr_ctx* c, const double* offsets, int32_t n_offsets) {
    if (!c) {
        g_thread_error = "corr_set_offsets: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] { set_offsets(c, offsets, n_offsets); });
}

int corr_eval_slices(corr_ctx* c, const double* quat_wxyz, int64_t n_rot, const corr_slices_out* out) {
    if (!c) {
        g_thread_error = "corr_eval_slices: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] {
        if (!out) fail(CORR_EINVAL, "out is NULL");
        EvalOut o;
        o.scores = out->scores;
        o.peak_val = out->peak_val;
        o.peak_idx = out->peak_idx;
        o.mask = out->obstacle;
        o.count = out->obstacle_count;
        o.thr = out->threshold;
        std::vector<const float2*> fas;
        for (const Slice& sl : c->slices) fas.push_back(sl.fa);
        if (fas.empty()) fas.push_back(c->fa);
        eval_entry(c, quat_wxyz, n_rot, fas, o);
    });
}

int corr_spectrum(corr_ctx* c, int32_t which, const double* quat_wxyz, float* out_dev) {
    if (!c) {
        g_thread_error = "corr_spectrum: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] {
        if (which != 0 && which != 1) fail(CORR_EINVAL, "which must be 0 (A) or 1 (B)");
        if (c->lifted) fail(CORR_EUNSUPPORTED, "corr_spectrum with CORR_LIFTED_SCORE: a slice has no single shape spectrum");
        join_a(c);
        if (!out_dev) fail(CORR_EINVAL, "out_dev is NULL");
        static const double ident[4] = {1, 0, 0, 0};
        const double* q = which == 0 ? ident : quat_wxyz;
        validate_quats(q, 1);
        const Shape& s = which == 0 ? c->A : c->B;
        stage_quats(c, q, 1);
        run_spectrum_stages(c, s, c->ws->quats, 1);
        stage(c, CORR_STAGE_FFT_Z_SPECTRUM, "fft z spectrum", [&] {
            return corr::launch_fft_z_spectrum(c->g, reinterpret_cast<float2*>(c->ws->buf0), 1, s.ex.q,
                                               occupancy(c, s), s.vtab, c->deconv,
                                               reinterpret_cast<float2*>(out_dev), c->twm, c->stream);
        });
    });
}

int corr_info(const corr_ctx* c, corr_info_t* out) {
    if (!c || !out) {
        g_thread_error = "corr_info: NULL argument";
        return CORR_EINVAL;
    }
    out->n = c->g.n;
    out->m = c->g.m;
    out->kb_width = c->g.w;
    out->q_a = c->A.ex.q;
    out->q_b = c->B.ex.q;
    out->n_a = c->A.n;
    out->n_b = c->B.n;
    out->batch = c->slots_eff > 0 ? c->slots_eff : c->ws->slots;
    out->workspace_bytes =
        (int64_t)(c->mem.bytes + (c->own_ws ? c->ws->mem.bytes : 0) + (c->ws_a ? c->ws_a->mem.bytes : 0));
    out->beta = c->g.beta;
    out->radius_err_a = c->A.ex.err;
    out->radius_err_b = c->B.ex.err;
    return CORR_OK;
}

int corr_profile(corr_ctx* c, int32_t enable) {
    if (!c) {
        g_thread_error = "corr_profile: NULL context";
        return CORR_EINVAL;
    }
    c->profiling = enable != 0;
    return CORR_OK;
}

int corr_profile_read(corr_ctx* c, double* ms, int64_t* launches, int32_t n_stages) {
    if (!c) {
        g_thread_error = "corr_profile_read: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] {
        if (n_stages < 0 || (n_stages > 0 && (!ms || !launches))) fail(CORR_EINVAL, "bad output arrays");
        for (int i = 0; i < n_stages; ++i) {
            ms[i] = 0;
            launches[i] = 0;
        }
        join_a(c);  // marks recorded on the side stream complete before a_done
        hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
        for (auto& mk : c->marks) {
            float t = 0;
            hip_check(hipEventElapsedTime(&t, mk.a, mk.b), "hipEventElapsedTime");
            if (mk.stage < n_stages) {
                ms[mk.stage] += t;
                launches[mk.stage] += 1;
            }
            c->spare.push_back(mk.a);
            c->spare.push_back(mk.b);
        }
        c->marks.clear();
    });
}

namespace {

// Add a workspace's spreading work record into out[3] and clear it (the
// stream that used it has drained).
void take_work(corr::Workspace* w, hipStream_t st, int64_t* out) {
    if (!w || !w->work) return;
    unsigned long long v[3] = {0, 0, 0};
    hip_check(hipMemcpy(v, w->work, sizeof v, hipMemcpyDeviceToHost), "work record D2H");
    for (int k = 0; k < 3; ++k) out[k] += (int64_t)v[k];
    hip_check(hipMemsetAsync(w->work, 0, sizeof v, st), "hipMemsetAsync");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

}  // namespace

int corr_spread_work(corr_ctx* c, int64_t* out) {
    if (!c) {
        g_thread_error = "corr_spread_work: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] {
        if (!out) fail(CORR_EINVAL, "out is NULL");
        out[0] = out[1] = out[2] = 0;
        join_a(c);  // A's side-stream passes complete before a_done
        hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
        if (c->own_ws) take_work(c->ws, c->stream, out);
        take_work(c->ws_a, c->stream, out);
    });
}

int corr_pass_info(corr_ctx* c, corr_pass_t* out) {
    if (!c) {
        g_thread_error = "corr_pass_info: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] {
        if (!out) fail(CORR_EINVAL, "out is NULL");
        const int nty = corr::spread_tiles(c->g);
        corr_pass_t r{};
        r.rotations = c->last_S;
        r.q = c->last_q;
        r.m = c->g.m;
        r.tile_rows = c->g.m / nty;
        r.knots = c->last_nk;
        r.tiles = (int64_t)c->last_S * c->g.m * nty;
        if (r.tiles > 0 && r.knots > 0) {
            std::vector<unsigned char> live((size_t)r.tiles);
            join_a(c);
            hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
            hip_check(hipMemcpy(live.data(), c->last_ws->tile_live, live.size(), hipMemcpyDeviceToHost),
                      "tile flags D2H");
            for (int64_t row = 0; row < (int64_t)c->last_S * c->g.m; ++row) {
                int64_t n = 0;
                for (int t = 0; t < nty; ++t) n += live[(size_t)row * nty + t] != 0;
                r.live_tiles += n;
                r.live_rows += n > 0;
            }
        }
        *out = r;
    });
}

namespace {

// Grow g to at least `bytes` (after the stream has drained its last users).
void* grow(corr_ctx* c, corr_ctx::Grown& g, size_t bytes) {
    if (bytes <= g.cap) return g.p;
    hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (g.p) (void)hipFree(g.p);
    g.p = nullptr;
    g.cap = 0;
    if (hipMalloc(&g.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        g.p = nullptr;
        fail(CORR_ENOMEM, "hipMalloc(%zu) for a query", bytes);
    }
    g.cap = bytes;
    return g.p;
}

// Half-space modes with |m|^2 <= r2 and |m_d| < n/2, in shell order (|m|^2, then
// mz, my, mx); returns the full-sphere count (m and -m).
int64_t query_modes(int n, int32_t r2, std::vector<int>& out) {
    const int h = n / 2 - 1;
    struct Md { int m2, mz, my, mx; };
    std::vector<Md> v;
    for (int mz = -h; mz <= h; ++mz)
        for (int my = -h; my <= h; ++my)
            for (int mx = 0; mx <= h; ++mx) {
                const int m2 = mx * mx + my * my + mz * mz;
                if (m2 > r2) continue;
                const bool half = mx > 0 || (mx == 0 && (my > 0 || (my == 0 && mz >= 0)));
                if (half) v.push_back({m2, mz, my, mx});
            }
    std::sort(v.begin(), v.end(), [](const Md& a, const Md& b) {
        if (a.m2 != b.m2) return a.m2 < b.m2;
        if (a.mz != b.mz) return a.mz < b.mz;
        if (a.my != b.my) return a.my < b.my;
        return a.mx < b.mx;
    });
    out.resize(v.size());
    for (size_t i = 0; i < v.size(); ++i)
        out[i] = (v[i].mx + 512) | ((v[i].my + 512) << 10) | ((v[i].mz + 512) << 20);
    return 2 * (int64_t)v.size() - 1;
}

}  // namespace

int corr_query(corr_ctx* c, const double* quat_wxyz, const double* t_host, int64_t n_t, int32_t mode_radius2,
               float* out_dev, int64_t* n_modes) {
    if (!c) {
        g_thread_error = "corr_query: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] {
        if (n_t < 0 || n_t > INT32_MAX) fail(CORR_EINVAL, "n_t = %lld; allowed 0..2^31-1", (long long)n_t);
        if (mode_radius2 < 0) fail(CORR_EINVAL, "mode_radius2 must be >= 0");
        if (n_t > 0 && (!t_host || !out_dev)) fail(CORR_EINVAL, "NULL translations or output");
        if (c->lifted) fail(CORR_EUNSUPPORTED, "queries with CORR_LIFTED_SCORE are not available");
        validate_quats(quat_wxyz, 1);
        for (int64_t i = 0; i < 3 * n_t; ++i)
            if (!std::isfinite(t_host[i])) fail(CORR_EINVAL, "translation %lld is not finite", (long long)(i / 3));
        join_a(c);  // F_A is read below
        const Geom& g = c->g;
        const int32_t full = 3 * (g.n / 2 - 1) * (g.n / 2 - 1);
        const int32_t r2 = std::min(mode_radius2, full);
        if (r2 != c->q_r2) {
            std::vector<int> modes;
            c->q_full = query_modes(g.n, r2, modes);
            void* d = grow(c, c->q_modes, sizeof(int) * modes.size());
            hip_check(hipMemcpyAsync(d, modes.data(), sizeof(int) * modes.size(), hipMemcpyHostToDevice, c->stream),
                      "mode list H2D");
            hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
            c->q_nm = (int)modes.size();
            c->q_r2 = r2;
        }
        if (n_modes) *n_modes = c->q_full;
        if (n_t == 0) return;
        const Shape& B = c->B;
        const int nm = c->q_nm;
        const corr::QueryPlan qp = corr::query_plan(nm, B.n, n_t);
        auto* part = static_cast<float2*>(grow(c, c->q_part, sizeof(float2) * nm * (size_t)qp.chunks));
        auto* tpart = static_cast<float*>(grow(c, c->q_tpart, sizeof(float) * (size_t)n_t * qp.mblocks));
        auto* P = static_cast<float2*>(grow(c, c->q_P, sizeof(float2) * nm));
        auto* dq = static_cast<double*>(grow(c, c->q_quat, sizeof(double) * 4));
        auto* dt = static_cast<double*>(grow(c, c->q_t, sizeof(double) * 3 * (size_t)n_t));
        // the caller's arrays are copied into pinned staging before returning
        const size_t need = 4 + 3 * (size_t)n_t;
        if (c->q_done) hip_check(hipEventSynchronize(c->q_done), "event sync");
        else hip_check(hipEventCreateWithFlags(&c->q_done, hipEventDisableTiming), "hipEventCreate");
        if (need > c->q_host_cap) {
            if (c->q_host) (void)hipHostFree(c->q_host);
            c->q_host = nullptr;
            c->q_host_cap = 0;
            hip_check(hipHostMalloc((void**)&c->q_host, sizeof(double) * need, hipHostMallocDefault), "hipHostMalloc");
            c->q_host_cap = need;
        }
        std::memcpy(c->q_host, quat_wxyz, sizeof(double) * 4);
        std::memcpy(c->q_host + 4, t_host, sizeof(double) * 3 * n_t);
        hip_check(hipMemcpyAsync(dq, c->q_host, sizeof(double) * 4, hipMemcpyHostToDevice, c->stream), "quat H2D");
        hip_check(hipMemcpyAsync(dt, c->q_host + 4, sizeof(double) * 3 * n_t, hipMemcpyHostToDevice, c->stream),
                  "translations H2D");
        hip_check(hipEventRecord(c->q_done, c->stream), "hipEventRecord");
        stage(c, CORR_STAGE_QUERY, "query", [&] {
            return corr::launch_query(g, qp, static_cast<const int*>(c->q_modes.p), nm, dq, B.pos, B.wts, B.n,
                                      B.ex.q, B.vtab, c->box, part, c->fa, P, dt, n_t, tpart, out_dev, c->stream);
        });
    });
}

// ---------------------------------------------------------------------------
// corr_query_noalloc: corr_query without any allocation.  Its device buffers
// (mode list, rotation, translations and the three partial-sum arrays of the
// query kernels) are carved out of one file-scope device array, `scratch`, of
// kNoAllocScratch bytes, which each GPU the library runs on holds until the
// process ends.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is taken once per device with
// hipGetSymbolAddress (that device current) and only that address is used.
// The host side works in fixed static arrays under a mutex, so the call makes
// no device, pinned or heap allocation.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr size_t kNoAllocScratch = (size_t)32 << 20;  // bytes of scratch per device
constexpr int kNoAllocModes = 1 << 16;                 // half-space modes per call
constexpr int kNoAllocDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

std::mutex g_noalloc_mu;                      // guards everything below
void* g_scratch_dev[kNoAllocDevices] = {};    // scratch's device address per device
uint64_t g_mode_keys[kNoAllocModes];          // (|m|^2, mz, my, mx) sort keys
int g_mode_list[kNoAllocModes];               // packed modes, as query_modes

// Device address of `scratch` on `dev` (looked up once, with dev current).
void* scratch_on(int dev) {
    if (dev < 0 || dev >= kNoAllocDevices) fail(CORR_EUNSUPPORTED, "device %d: no scratch slot", dev);
    if (g_scratch_dev[dev]) return g_scratch_dev[dev];
    int cur = 0;
    hip_check(hipGetDevice(&cur), "hipGetDevice");
    if (cur != dev) hip_check(hipSetDevice(dev), "hipSetDevice");
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    hip_check(e, "hipGetSymbolAddress (scratch)");
    if (!ptr) fail(CORR_EHIP, "hipGetSymbolAddress (scratch): null address");
    g_scratch_dev[dev] = ptr;
    return ptr;
}

// The half-space modes of query_modes, in the same shell order, into
// g_mode_list without allocating; returns the count (fails past the cap) and
// the full-sphere count in *full.
int query_modes_static(int n, int32_t r2, int64_t* full) {
    const int h = n / 2 - 1;
    int rad = 0;
    while (rad < h && (int64_t)(rad + 1) * (rad + 1) <= r2) ++rad;
    int nm = 0;
    for (int mz = -rad; mz <= rad; ++mz)
        for (int my = -rad; my <= rad; ++my)
            for (int mx = 0; mx <= rad; ++mx) {
                const int m2 = mx * mx + my * my + mz * mz;
                if (m2 > r2) continue;
                if (!(mx > 0 || (mx == 0 && (my > 0 || (my == 0 && mz >= 0))))) continue;
                if (nm == kNoAllocModes)
                    fail(CORR_EUNSUPPORTED, "mode_radius2 = %d keeps more than %d half-space modes, the most "
                                            "corr_query_noalloc takes", r2, kNoAllocModes);
                g_mode_keys[nm++] = ((uint64_t)m2 << 30) | ((uint64_t)(mz + 512) << 20) |
                                    ((uint64_t)(my + 512) << 10) | (uint64_t)(mx + 512);
            }
    std::sort(g_mode_keys, g_mode_keys + nm);  // in place: (|m|^2, mz, my, mx)
    for (int i = 0; i < nm; ++i) {
        const uint64_t k = g_mode_keys[i];
        g_mode_list[i] = (int)(k & 1023) | ((int)((k >> 10) & 1023) << 10) | ((int)((k >> 20) & 1023) << 20);
    }
    *full = 2 * (int64_t)nm - 1;
    return nm;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

int corr_query_noalloc(corr_ctx* c, const double* quat_wxyz, const double* t_host, int64_t n_t,
                       int32_t mode_radius2, float* out_dev, int64_t* n_modes) {
    if (!c) {
        g_thread_error = "corr_query_noalloc: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] {
        if (n_t < 0 || n_t > INT32_MAX) fail(CORR_EINVAL, "n_t = %lld; allowed 0..2^31-1", (long long)n_t);
        if (mode_radius2 < 0) fail(CORR_EINVAL, "mode_radius2 must be >= 0");
        if (n_t > 0 && (!t_host || !out_dev)) fail(CORR_EINVAL, "NULL translations or output");
        if (c->lifted) fail(CORR_EUNSUPPORTED, "queries with CORR_LIFTED_SCORE are not available");
        validate_quats(quat_wxyz, 1);
        for (int64_t i = 0; i < 3 * n_t; ++i)
            if (!std::isfinite(t_host[i])) fail(CORR_EINVAL, "translation %lld is not finite", (long long)(i / 3));
        const Geom& g = c->g;
        const int32_t full = 3 * (g.n / 2 - 1) * (g.n / 2 - 1);
        const int32_t r2 = std::min(mode_radius2, full);
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        int64_t nfull = 0;
        const int nm = query_modes_static(g.n, r2, &nfull);
        if (n_modes) *n_modes = nfull;
        if (n_t == 0) return;
        const Shape& B = c->B;
        const corr::QueryPlan qp = corr::query_plan(nm, B.n, n_t);
        // scratch layout: modes, rotation, translations, chunk sums, mode
        // products, translation partial sums (each 256-byte aligned)
        const size_t b_modes = align256(sizeof(int) * nm), b_quat = align256(sizeof(double) * 4),
                     b_t = align256(sizeof(double) * 3 * (size_t)n_t),
                     b_part = align256(sizeof(float2) * (size_t)nm * qp.chunks), b_P = align256(sizeof(float2) * nm),
                     b_tpart = align256(sizeof(float) * (size_t)n_t * qp.mblocks);
        const size_t need = b_modes + b_quat + b_t + b_part + b_P + b_tpart;
        if (need > kNoAllocScratch)
            fail(CORR_EUNSUPPORTED, "this query needs %zu bytes of scratch; corr_query_noalloc holds %zu per device "
                                    "(use fewer modes or translations, or corr_query)", need, kNoAllocScratch);
        auto* base = static_cast<unsigned char*>(scratch_on(c->device));
        int* d_modes = reinterpret_cast<int*>(base);
        double* dq = reinterpret_cast<double*>(base + b_modes);
        double* dt = reinterpret_cast<double*>(base + b_modes + b_quat);
        auto* part = reinterpret_cast<float2*>(base + b_modes + b_quat + b_t);
        auto* P = reinterpret_cast<float2*>(base + b_modes + b_quat + b_t + b_part);
        auto* tpart = reinterpret_cast<float*>(base + b_modes + b_quat + b_t + b_part + b_P);
        join_a(c);  // F_A is read below
        // pageable copies: each returns once its source may be reused; every
        // kernel below writes what it later reads, so nothing needs clearing
        hip_check(hipMemcpyAsync(d_modes, g_mode_list, sizeof(int) * nm, hipMemcpyHostToDevice, c->stream),
                  "mode list H2D");
        hip_check(hipMemcpyAsync(dq, quat_wxyz, sizeof(double) * 4, hipMemcpyHostToDevice, c->stream), "quat H2D");
        hip_check(hipMemcpyAsync(dt, t_host, sizeof(double) * 3 * n_t, hipMemcpyHostToDevice, c->stream),
                  "translations H2D");
        hip_check(corr::launch_query(g, qp, d_modes, nm, dq, B.pos, B.wts, B.n, B.ex.q, B.vtab, c->box, part, c->fa, P,
                                     dt, n_t, tpart, out_dev, c->stream),
                  "query");
    });
}

int corr_raster_eval(corr_ctx* c, const double* quat_wxyz, int64_t n_rot, int32_t* counts_dev) {
    if (!c) {
        g_thread_error = "corr_raster_eval: NULL context";
        return CORR_EINVAL;
    }
    return guarded(c, [&] {
        if (n_rot < 0) fail(CORR_EINVAL, "n_rot = %lld", (long long)n_rot);
        if (n_rot == 0) return;
        if (!counts_dev) fail(CORR_EINVAL, "counts_dev is NULL");
        validate_quats(quat_wxyz, n_rot);
        join_a(c);
        const Geom& g = c->g;
        const size_t n3 = (size_t)g.n * g.n * g.n;
        auto* grid = static_cast<double2*>(grow(c, c->r_grid, sizeof(double2) * n3));
        auto* dq = static_cast<double*>(grow(c, c->r_quat, sizeof(double) * 4 * (size_t)n_rot));
        if (!c->r_tw.p) {
            std::vector<double2> tw(g.n);
            for (int j = 0; j < g.n; ++j)
                tw[j] = make_double2(std::cos(2.0 * M_PI * j / g.n), -std::sin(2.0 * M_PI * j / g.n));
            auto* d = static_cast<double2*>(grow(c, c->r_tw, sizeof(double2) * g.n));
            upload(d, tw.data(), sizeof(double2) * g.n, c->stream);
        }
        upload(dq, quat_wxyz, sizeof(double) * 4 * (size_t)n_rot, c->stream);
        const double h = c->box / g.n;
        for (int64_t r = 0; r < n_rot; ++r)
            stage(c, CORR_STAGE_RASTER, "raster", [&] {
                return corr::launch_raster_counts(g.n, h, c->origin, c->A.pos, c->A.rad, c->A.n, c->B.pos, c->B.rad,
                                                  c->B.n, dq + 4 * r, static_cast<const double2*>(c->r_tw.p), grid,
                                                  counts_dev + r * n3, c->stream);
            });
    });
}

struct corr_batch {
    hipStream_t stream = nullptr;
    std::vector<corr_ctx*> pairs;
    corr::Workspace ws;
    bool graph = false;  // replay whole batch evaluations as one captured hipGraph
    GraphState gs;
    std::string err = "no error";
};

int corr_batch_create(const corr_pair* pairs, int32_t n_pairs, int32_t slots, void* hip_stream, corr_batch** out) {
    corr_batch* b = nullptr;
    int rc = guarded(nullptr, [&] {
        if (!out) fail(CORR_EINVAL, "out is NULL");
        *out = nullptr;
        if (n_pairs < 1 || !pairs) fail(CORR_EINVAL, "need n_pairs >= 1 pairs");
        if (slots < 0 || slots > 256) fail(CORR_EINVAL, "slots = %d; allowed 0..256", slots);
        b = new corr_batch();
        b->stream = static_cast<hipStream_t>(hip_stream);
        corr::WsReq r;
        for (int p = 0; p < n_pairs; ++p) {
            char who[64];
            snprintf(who, sizeof who, "pair %d: ", p);
            const corr_pair& pr = pairs[p];
            b->pairs.push_back(plan_pair(pr.A, pr.nA, pr.B, pr.nB, &pr.grid, hip_stream, who));
            r.merge(ws_req(b->pairs.back()));
        }
        if (slots == 0) {
            // rotations per pass chosen per pair, from an 8 GiB budget (at most
            // 64): every buffer is sized for the pair that needs most of it, and
            // each pair indexes the buffers by its own geometry
            corr::WsReq all;
            int qslots = 1;
            for (corr_ctx* c : b->pairs) {
                const corr::WsReq rp = ws_req(c);
                c->slots_eff = (int)std::max<size_t>(1, std::min<size_t>(64, ((size_t)8 << 30) / rp.slot_bytes()));
                all.merge(rp.scaled((size_t)c->slots_eff));
                qslots = std::max(qslots, c->slots_eff);
            }
            b->ws.allocate(1, all, b->stream, qslots);
        } else {
            // `slots` rotations per pass for the pair that needs most; a pair on a
            // smaller grid (or with fewer knots) packs more into the same buffers
            int qslots = slots;
            for (corr_ctx* c : b->pairs) {
                c->slots_eff = r.slots_for(ws_req(c), slots);
                qslots = std::max(qslots, c->slots_eff);
            }
            b->ws.allocate(slots, r, b->stream, qslots);
        }
        for (corr_ctx* c : b->pairs) {
            c->ws = &b->ws;
            c->own_ws = false;
            prepare_a(c);
        }
        *out = b;
    });
    if (rc != CORR_OK && b) corr_batch_destroy(b);
    return rc;
}

int corr_batch_eval(corr_batch* b, const double* quat_wxyz, const int64_t* rot_offsets, float* scores_dev,
                    const int64_t* score_offsets, float* peak_val_dev, int64_t* peak_idx_dev) {
    if (!b) {
        g_thread_error = "corr_batch_eval: NULL batch";
        return CORR_EINVAL;
    }
    corr_ctx* cur = nullptr;
    int rc = guarded(nullptr, [&] {
        const int np = (int)b->pairs.size();
        if (!rot_offsets) fail(CORR_EINVAL, "rot_offsets is NULL");
        if (rot_offsets[0] != 0) fail(CORR_EINVAL, "rot_offsets[0] must be 0");
        for (int p = 0; p < np; ++p)
            if (rot_offsets[p + 1] < rot_offsets[p]) fail(CORR_EINVAL, "rot_offsets must not decrease (pair %d)", p);
        if ((peak_val_dev == nullptr) != (peak_idx_dev == nullptr))
            fail(CORR_EINVAL, "peak_val_dev and peak_idx_dev must both be set or both be NULL");
        validate_quats(quat_wxyz, rot_offsets[np]);
        // every pair's outputs; with a graph, its rotations come from dq
        auto run = [&](const double* dq) {
            int64_t packed = 0;
            for (int p = 0; p < np; ++p) {
                corr_ctx* c = b->pairs[p];
                cur = c;
                const int64_t r0 = rot_offsets[p], nr = rot_offsets[p + 1] - rot_offsets[p];
                const int64_t n3 = (int64_t)c->g.n * c->g.n * c->g.n;
                EvalOut o;
                if (scores_dev) o.scores = scores_dev + (score_offsets ? score_offsets[p] : packed);
                packed += nr * n3;
                o.peak_val = peak_val_dev ? peak_val_dev + r0 : nullptr;
                o.peak_idx = peak_idx_dev ? peak_idx_dev + r0 : nullptr;
                eval_impl(c, dq ? nullptr : quat_wxyz + 4 * r0, nr, {c->fa}, o, dq ? dq + 4 * r0 : nullptr);
            }
        };
        if (!b->graph || rot_offsets[np] == 0) {
            run(nullptr);
            return;
        }
        const double* dq = graph_quats(b->gs, b->stream, quat_wxyz, rot_offsets[np]);
        std::vector<uint64_t> key = {2, (uint64_t)(uintptr_t)scores_dev, (uint64_t)(uintptr_t)peak_val_dev,
                                     (uint64_t)(uintptr_t)peak_idx_dev, score_offsets ? 1u : 0u};
        for (int p = 0; p <= np; ++p) key.push_back((uint64_t)rot_offsets[p]);
        if (score_offsets)
            for (int p = 0; p < np; ++p) key.push_back((uint64_t)score_offsets[p]);
        // a pair's launch shapes (its tuning) are part of what the graph holds
        for (corr_ctx* c : b->pairs) key.push_back(c->shape_gen);
        graph_launch(b->gs, b->stream, std::move(key), b->pairs, nullptr, [&] { run(dq); });
    });
    if (rc != CORR_OK) b->err = cur && cur->err != "no error" ? cur->err : g_thread_error;
    return rc;
}

int corr_batch_set_graph(corr_batch* b, int32_t enable) {
    if (!b) {
        g_thread_error = "corr_batch_set_graph: NULL batch";
        return CORR_EINVAL;
    }
    if (enable != 0 && enable != 1) {
        b->err = "corr_batch_set_graph: enable must be 0 or 1";
        return CORR_EINVAL;
    }
    b->graph = enable != 0;
    return CORR_OK;
}

int corr_batch_spread_work(corr_batch* b, int64_t* out) {
    if (!b || !out) {
        g_thread_error = "corr_batch_spread_work: NULL batch or output";
        return CORR_EINVAL;
    }
    int rc = guarded(nullptr, [&] {
        out[0] = out[1] = out[2] = 0;
        hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
        take_work(&b->ws, b->stream, out);
    });
    if (rc != CORR_OK) b->err = g_thread_error;
    return rc;
}

int corr_batch_profile(corr_batch* b, int32_t enable) {
    if (!b) {
        g_thread_error = "corr_batch_profile: NULL batch";
        return CORR_EINVAL;
    }
    for (corr_ctx* c : b->pairs) c->profiling = enable != 0;
    return CORR_OK;
}

int corr_batch_profile_read(corr_batch* b, double* ms, int64_t* launches, int32_t n_stages) {
    if (!b) {
        g_thread_error = "corr_batch_profile_read: NULL batch";
        return CORR_EINVAL;
    }
    if (n_stages < 0 || (n_stages > 0 && (!ms || !launches))) {
        b->err = "corr_batch_profile_read: bad output arrays";
        return CORR_EINVAL;
    }
    std::vector<double> pm((size_t)n_stages);
    std::vector<int64_t> pl((size_t)n_stages);
    for (int i = 0; i < n_stages; ++i) {
        ms[i] = 0;
        launches[i] = 0;
    }
    for (corr_ctx* c : b->pairs) {
        const int rc = corr_profile_read(c, pm.data(), pl.data(), n_stages);
        if (rc != CORR_OK) {
            b->err = c->err;
            return rc;
        }
        for (int i = 0; i < n_stages; ++i) {
            ms[i] += pm[i];
            launches[i] += pl[i];
        }
    }
    return CORR_OK;
}

int corr_batch_autotune(corr_batch* b, const double* quat_wxyz, const int64_t* rot_offsets, float* scores_dev,
                        const int64_t* score_offsets, float* peak_val_dev, int64_t* peak_idx_dev, int32_t reps,
                        int32_t* out7) {
    if (!b) {
        g_thread_error = "corr_batch_autotune: NULL batch";
        return CORR_EINVAL;
    }
    if (reps < 1 || reps > 100) {
        b->err = "corr_batch_autotune: reps must be in 1..100";
        return CORR_EINVAL;
    }
    // a candidate: spread_wgs and, for each grid size of the batch (largest
    // first), per column pass, for the bin group and for the tile height, the
    // rank of the value among each pair's choices (0 its default, 1 and 2 the
    // others where they exist)
    constexpr int kMaxGrids = 8;
    struct Cand {
        int wgs;
        int rank[kMaxGrids][6];
    };
    std::vector<corr_tuning> start;
    for (corr_ctx* c : b->pairs) start.push_back(get_tuning(c));
    std::vector<int> grids;  // distinct spreading grids, largest first
    for (corr_ctx* c : b->pairs)
        if (std::find(grids.begin(), grids.end(), c->g.m) == grids.end()) grids.push_back(c->g.m);
    std::sort(grids.begin(), grids.end(), std::greater<int>());
    std::vector<int> grid_of(b->pairs.size());
    for (size_t i = 0; i < b->pairs.size(); ++i)
        grid_of[i] = (int)(std::find(grids.begin(), grids.end(), b->pairs[i]->g.m) - grids.begin());
    if ((int)grids.size() > kMaxGrids) {  // grids are powers of two from 32 to 512: cannot happen
        b->err = "corr_batch_autotune: too many grid sizes";
        return CORR_EUNSUPPORTED;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = guarded(nullptr, [&] {
        hip_check(hipEventCreate(&e0), "hipEventCreate");
        hip_check(hipEventCreate(&e1), "hipEventCreate");
    });
    if (rc != CORR_OK) {
        b->err = g_thread_error;
        return rc;
    }
    auto apply = [&](const Cand& k) {
        for (size_t i = 0; i < b->pairs.size(); ++i) {
            corr_ctx* c = b->pairs[i];
            const int* rank = k.rank[grid_of[i]];
            corr_tuning t = start[i];
            t.spread_wgs = k.wgs;
            int32_t corr_tuning::*fields[4] = {&corr_tuning::cols_y, &corr_tuning::cols_z, &corr_tuning::cols_iy,
                                               &corr_tuning::pairs_ix};
            for (int p = 0; p < 4; ++p) {
                int ch[3];
                const int n = corr::col_choices(c->g.m, p, ch);
                t.*fields[p] = ch[rank[p] < n ? rank[p] : 0];
            }
            int bg[3];
            const int nb = corr::bin_choices(c->g.m, bg);
            t.bin_group = bg[rank[4] < nb ? rank[4] : 0];
            int tr[2];
            const int nt = corr::tile_choices(c->g.m, tr);
            t.tile_rows = tr[rank[5] < nt ? rank[5] : 0];
            set_tuning(c, t);
        }
    };
    float best_ms = INFINITY;
    Cand cur{};
    cur.wgs = start.empty() ? 1 : start[0].spread_wgs;
    auto timed = [&](const Cand& k) -> float {
        apply(k);
        auto unit = [&] {
            const int r = corr_batch_eval(b, quat_wxyz, rot_offsets, scores_dev, score_offsets, peak_val_dev,
                                          peak_idx_dev);
            if (r != CORR_OK) throw CorrError{r, b->err};
        };
        unit();  // untimed: first touch, graph capture
        float best = INFINITY;
        for (int r = 0; r < reps; ++r) {
            hip_check(hipEventRecord(e0, b->stream), "hipEventRecord");
            unit();
            hip_check(hipEventRecord(e1, b->stream), "hipEventRecord");
            hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            best = std::min(best, ms);
        }
        return best;
    };
    rc = guarded(nullptr, [&] {
        const int cus = b->pairs.empty() ? 1 : cu_count(b->pairs[0]);
        best_ms = timed(cur);
        for (int v : {cus, cus + cus / 2, 2 * cus}) {
            if (v == cur.wgs) continue;
            Cand k = cur;
            k.wgs = v;
            const float ms = timed(k);
            if (ms < best_ms) {
                best_ms = ms;
                cur = k;
            }
        }
        for (size_t gi = 0; gi < grids.size(); ++gi)
            for (int p = 0; p < 6; ++p)
                for (int r = 1; r < (p == 5 ? 2 : 3); ++r) {
                    Cand k = cur;
                    k.rank[gi][p] = r;
                    const float ms = timed(k);
                    if (ms < best_ms) {
                        best_ms = ms;
                        cur = k;
                    }
                }
        apply(cur);
        // the outputs hold an evaluation under the kept tuning
        const int r = corr_batch_eval(b, quat_wxyz, rot_offsets, scores_dev, score_offsets, peak_val_dev, peak_idx_dev);
        if (r != CORR_OK) throw CorrError{r, b->err};
        hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    });
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != CORR_OK) {
        (void)hipStreamSynchronize(b->stream);
        for (size_t i = 0; i < b->pairs.size(); ++i) {
            try {
                set_tuning(b->pairs[i], start[i]);
            } catch (...) {
            }
        }
        b->err = g_thread_error;
        return rc;
    }
    if (out7) {
        out7[0] = cur.wgs;
        for (int p = 0; p < 6; ++p) out7[1 + p] = cur.rank[0][p];  // the largest grid's
    }
    return CORR_OK;
}

int corr_batch_info(const corr_batch* b, int32_t pair, corr_info_t* out) {
    if (!b || pair < 0 || pair >= (int32_t)b->pairs.size()) {
        g_thread_error = "corr_batch_info: bad batch or pair index";
        return CORR_EINVAL;
    }
    return corr_info(b->pairs[pair], out);
}

int corr_batch_destroy(corr_batch* b) {
    if (!b) return CORR_OK;
    (void)hipStreamSynchronize(b->stream);
    for (corr_ctx* c : b->pairs) destroy_ctx(c);
    b->gs.release();
    b->ws.release();
    delete b;
    return CORR_OK;
}

const char* corr_batch_last_error(const corr_batch* b) { return b ? b->err.c_str() : g_thread_error.c_str(); }

int corr_destroy(corr_ctx* c) {
    destroy_ctx(c);
    return CORR_OK;
}

const char* corr_last_error(const corr_ctx* c) {
    return c ? c->err.c_str() : g_thread_error.c_str();
}

}  // extern "C"

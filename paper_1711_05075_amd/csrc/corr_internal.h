// Internal interface between the host side (corr_host.cpp) and the gfx950
// kernels (corr_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace corr {

// Sizes of one correlation grid.
//   n     translations per axis (the kept modes are |m_d| < n/2)
//   m     spreading grid per axis (sigma * n), a power of two
//   w     Kaiser-Bessel window width in spreading cells
//   m2n   entries of a ball-transform table: |m|^2 = 0 .. 3 (n/2 - 1)^2
struct Geom {
    int n = 0, m = 0, w = 0, half = 0, m2n = 0;
    float beta = 0.f;         // window shape
    float inv_i0beta = 0.f;   // 1 / I0(beta): window normalised to 1 at its centre
    double inv_hf = 0.0;      // 1 / spreading-cell size
    int spread_wgs = 0;       // workgroups of the persistent spreading pass (two per CU)
    // column batch of each column-FFT pass (0: the pass's default width; else
    // the default, half of it or twice it, see col_choices): forward y, z
    // passes, inverse y and slice products, inverse x (line pairs)
    int cols_y = 0, cols_z = 0, cols_iy = 0, pairs_ix = 0;
    // y-group of the sort keys (the bins of spreading), in cells: 0 for
    // bin_ygroup(m), else one of bin_choices(m)
    int bin_group = 0;
    // rows of a spreading tile: 0 for the default at m, else one of
    // tile_choices(m)
    int tile_rows = 0;
};

// Widths a column pass may take at spreading-grid size m: out[0] is the
// default, then the others (half and twice the default where the pass allows
// them).  pass: 0 forward y, 1 z passes, 2 inverse y, 3 inverse x.  Returns
// the count (1..3), 0 for an unsupported m or pass.
int col_choices(int m, int pass, int out[3]);

// Which parts of a rotation's spreading grid hold knots.  z row z is live iff
// some knot's z-window reaches it, which the z-sorted bin starts tell directly;
// y tile t of a live row is live iff some knot's window reaches it, which the
// spreading pass records in tile_live.  The passes after it read only live rows
// and tiles: the others are zero by construction and are never written.
struct Occupancy {
    const int* bin_start = nullptr;         // [S][keys + 1] first sorted knot of each key
    unsigned char* tile_live = nullptr;     // [S][m][spread_tiles(g)]
    int64_t nk = 0;                         // knots per rotation
};
// y tiles per z row of the spreading pass, and the most any tile height of
// tile_choices gives (the size the tile arrays are allocated for).
int spread_tiles(const Geom& g);
int spread_tiles_max(const Geom& g);
// Rows a spreading tile may take at m: out[0] the default, out[1] half of it.
// Returns the count.
int tile_choices(int m, int out[2]);
// ints of a spreading pass's plan counters; its live-tile list holds
// plan_buckets() * S * m * spread_tiles(g) ints.
int plan_words();
constexpr int plan_buckets() { return 8; }

// ---- table builders (FP64 on the device) ---------------------------------
hipError_t launch_deconv_tables(const Geom& g, double box, const double origin[3],
                                double* d_deconv /*[n]*/, double2* d_phase /*[3][n]*/,
                                hipStream_t st);
// Per-ball kernel table: K(k; r) = Bhat(k; r + r0) - lam Bhat(k; r) expanded on
// the radius basis (r0 = lam = 0: the ball transform), normalised by rref^3.
hipError_t launch_ball_table(const Geom& g, double dk, const double* d_nodes, const double* d_basis,
                             int p, int q, double rref, double r0, double lam,
                             float* d_vtab /*[q][m2n]*/, hipStream_t st);

// ---- pipeline stages -----------------------------------------------------
// Knots are sorted by key = z-cell * (m / ygroup) + y-cell / ygroup, with
// y-groups of ygroup(m) cells by default, chosen so that there are at most
// 16384 keys (m = 256: groups of 4 cells, so that a tile of 8 rows and a
// window of 6 reads about 16 candidate cells for the 13 that reach it).  The
// tuning may take half or twice that group where the key count stays within
// [1024, 32768] (bin_choices); a rotation's key starts always have room for
// the finest choice.
constexpr int bin_ygroup(int m) { return m * m / 16384 > 1 ? m * m / 16384 : 1; }
constexpr int bin_ygroup_min(int m) {
    return bin_ygroup(m) > 1 && m * m / (bin_ygroup(m) / 2) <= 32768 ? bin_ygroup(m) / 2 : bin_ygroup(m);
}
constexpr int bin_keys_max(int m) { return m * (m / bin_ygroup_min(m)); }
// Groups a grid of spreading size m may take: out[0] the default, then half
// and twice it where allowed.  Returns the count (1..3).
int bin_choices(int m, int out[3]);
// The group a geometry uses.
inline int bin_group(const Geom& g) { return g.bin_group > 0 ? g.bin_group : bin_ygroup(g.m); }
// a0, binned: rotate, place (d_rec [S][nk]: packed cell and the FP32 offsets
// from it), and each knot's rank among the knots of its key from atomic
// counters (d_counts [S][keys], zero on entry); then the scan of the counts
// into d_bin_start [S][keys + 1], which clears them.  Also clears the
// live-tile plan's counters d_plan.
hipError_t launch_rotate_bin(const Geom& g, const double* d_quats, int S, const double* d_pos, int64_t nk,
                             int4* d_rec, int* d_rank, int* d_counts, int* d_bin_start, int* d_plan, hipStream_t st);
// The scatter of every knot into sorted order (its cell, its window weights
// along x, y and z evaluated from its offsets, its q component weights), and
// the live-tile plan: tiles that no knot's window can reach are marked dead in
// occ.tile_live and the others are listed in d_list by the size of their
// candidate sets (d_plan: bucket sizes and the spreading pass's work counter).
hipError_t launch_scatter_plan(const Geom& g, int S, int q, const Occupancy& occ, const int4* d_rec,
                               const float* d_wts, const int* d_rank, int* d_scell, float* d_skbw, float* d_swts,
                               int* d_plan, int* d_list, hipStream_t st);
// a1 + a2 (x): gather-spreading of the sorted knots fused with the x transform;
// writes [S][q][z][y][mx] without a spreading grid in HBM.
// Sums are exact 64-bit fixed point of 32-bit addends; fix_scale is a power of
// two with fix_scale * max_{i,c} |wts[c][i]| <= 2^30.
// Runs g.spread_wgs persistent workgroups over the plan's tiles; a listed tile
// that no knot reaches only records that in occ.tile_live.  Adds its work to
// d_work[3]: bytes of kept x modes written (live tiles only), bytes of sorted
// knot records (cell, window weights, component weights) of the pass, and 1
// launch.
hipError_t launch_spread_fftx(const Geom& g, int S, const Occupancy& occ, int* d_plan, const int* d_list,
                              const int* d_scell, const float* d_skbw, const float* d_swts, int q, float fix_scale,
                              float2* d_out, const float2* d_twm, unsigned long long* d_work, hipStream_t st);
// Largest dynamic LDS any stage asks for.
size_t max_lds_bytes(const Geom& g, int qmax);
// a2: pruned forward y pass of S rotations x q components (live rows only).
hipError_t launch_fft_y(const Geom& g, int S, int q, const Occupancy& occ, const float2* d_in, float2* d_out,
                        const float2* d_twm, hipStream_t st);
// a2 (z) + a3: z transform of every component, the radius-expansion sum with the
// ball-transform table, and the deconvolution; writes the shape spectrum.  With
// d_deconv NULL it writes the sums without the deconvolution (for
// launch_product_ifft_z).
hipError_t launch_fft_z_spectrum(const Geom& g, const float2* d_in, int S, int q, const Occupancy& occ,
                                 const float* d_vtab, const double* d_deconv, float2* d_spec,
                                 const float2* d_twm, hipStream_t st);
// a2 (z) + a3 + a4 + first inverse pass of a5: as above for the rotated shape,
// times the fixed shape's spectrum, the origin phase and 1/L^3, then the
// inverse z transform.
hipError_t launch_fft_z_product(const Geom& g, const float2* d_in, int S, int q, const Occupancy& occ,
                                const float* d_vtab, const double2* d_phase, const float2* d_fa,
                                float2* d_out, const float2* d_twm, const float2* d_twn,
                                hipStream_t st);
// a4 + first inverse pass of a5 for one more fixed spectrum d_fa, from the
// rotated shape's z sums d_acc [S][n][n][half]: the product and inverse z of
// launch_fft_z_product, bit for bit.
hipError_t launch_product_ifft_z(const Geom& g, const float2* d_acc, int S, const double2* d_phase,
                                 const float2* d_fa, float2* d_out, const float2* d_twn, hipStream_t st);
// ---- the lifted score (4D cone correlation sliced at heights h) -------------
// d_tab [qa][qb][m2n] = What(dk sqrt(m2); a_p + b_p' - h) at the two shapes'
// radius nodes d_na [qa], d_nb [qb] (FP64, stored as float).
hipError_t launch_lift_table(const Geom& g, double dk, const double* d_na, int qa, const double* d_nb, int qb,
                             double h, float* d_tab, hipStream_t st);
// z transform of every component kept apart: d_out [S][q][n][n][half], times
// the deconvolution if d_deconv is not NULL.
hipError_t launch_fft_z_components(const Geom& g, const float2* d_in, int S, int q, const Occupancy& occ,
                                   const double* d_deconv, float2* d_out, const float2* d_twm, hipStream_t st);
// d_h [qb][n][n][half] = sum_p d_ga[p] * d_tab[p][.][|m|^2] per mode.
hipError_t launch_lift_h(const Geom& g, const float2* d_ga, int qa, const float* d_tab, int qb, float2* d_h,
                         hipStream_t st);
// product sum_c d_h[c] conj(d_comps[s][c]) times the shift and deconvolution
// factor, then inverse z: d_out [S][n][n][half].
hipError_t launch_lift_product_ifft_z(const Geom& g, const float2* d_comps, int S, int q, const double2* d_phase,
                                      const float2* d_h, float2* d_out, const float2* d_twn, hipStream_t st);

// a5: inverse y (d_in == d_out allowed), then inverse x (half-complex to real)
// with per-block peaks and, for the obstacle predicate score > thr, the bit
// mask d_mask [S][n^3 / 32] (NULL: not written) and per-block counts d_pcnt
// (NULL: not counted).  d_scores NULL: scores not written.
hipError_t launch_ifft_y(const Geom& g, const float2* d_in, int S, float2* d_out,
                         const float2* d_twn, hipStream_t st);
int ifft_x_blocks(const Geom& g);
// The most inverse-x blocks any allowed pairs_ix gives (workspace sizing).
int ifft_x_blocks_max(const Geom& g);
hipError_t launch_ifft_x(const Geom& g, const float2* d_in, int S, float* d_scores, unsigned* d_mask, float thr,
                         float* d_pval, int* d_pidx, int* d_pcnt, const float2* d_twn, hipStream_t st);
// Per rotation: peak (d_peak_val, d_peak_idx; NULL: skipped) and obstacle count
// (d_count; NULL: skipped) from the inverse-x blocks.
hipError_t launch_peak_final(const float* d_pval, const int* d_pidx, const int* d_pcnt, int S, int nblocks,
                             float* d_peak_val, int64_t* d_peak_idx, int64_t* d_count, hipStream_t st);

// ---- uniform-rasterization baseline (raster_kernels.hip) ------------------
// Voxel-overlap counts of one rotation: both shapes sampled on the n^3 grid
// (A at origin + h u, B turned by d_quat at h v, v signed), the grids
// correlated by an FP64 FFT in d_grid (n^3 double2, overwritten), and
// d_counts [n^3] (int32, [tz][ty][tx]) = sum_u a(u) b(u - t), exact.
// d_tw [n] = exp(-2 pi i j / n) in FP64.
hipError_t launch_raster_counts(int n, double h, const double origin[3], const double* d_pos_a, const double* d_rad_a,
                                int64_t na, const double* d_pos_b, const double* d_rad_b, int64_t nb,
                                const double* d_quat, const double2* d_tw, double2* d_grid, int32_t* d_counts,
                                hipStream_t st);

// ---- single-configuration query -------------------------------------------
// d_modes: nm packed modes (mx + 512) | (my + 512) << 10 | (mz + 512) << 20 of the
// half space.  Scratch: d_part float2 [chunks][nm], d_P float2 [nm], d_tpart
// float [n_t][mblocks].
struct QueryPlan {
    int kch = 256, chunks = 1;  // knots per NDFT chunk, chunks
    int mblocks = 1, mper = 1;  // mode blocks per translation sum, modes per block
};
QueryPlan query_plan(int nm, int64_t nk, int64_t n_t);
hipError_t launch_query(const Geom& g, const QueryPlan& qp, const int* d_modes, int nm, const double* d_quat,
                        const double* d_pos, const float* d_wts, int64_t nk, int q, const float* d_vtab, double box,
                        float2* d_part, const float2* d_fa, float2* d_P, const double* d_t, int64_t n_t,
                        float* d_tpart, float* d_out, hipStream_t st);

}  // namespace corr

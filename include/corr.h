/*
 * corr.h -- C ABI of the MI355X ball-union correlation library (libcorr.so).
 *
 * Computes the correlation score of two shapes, each a union of weighted balls,
 * for every translation of a 3D grid and for many rotations:
 *
 *     s(R, t) = < f_A , f_{(R,t)B} >  =  sum_i sum_j c_i d_j vol( B(x_i, r_i) & B(R y_j + t, rho_j) )
 *
 * (Behandish & Ilies, CAD 2016: the correlation function of Sec. 3.1
 * eq. eq_relg_0 for defining functions that are sums of ball indicators,
 * Sec. 2.1 eq. eq_un and Sec. 2.2 eq. eq_Psum; the motion acts as x -> R x + t,
 * App. B).  It is evaluated by the Fourier route of Sec. 3.2 eq. eq_ccghat:
 * per-shape spectra by a nonequispaced FFT of the knots (Sec. 2.5
 * eq. eq_rhoPhat) weighted by the ball transform, their product, and an inverse
 * FFT onto the translation grid.  The result is the band-limited score: only
 * the modes k = 2 pi m / L with |m_d| < n/2 of the L-periodic score are kept.
 *
 * Conventions
 *  - Balls are {x, y, z, r, w}: centre, radius (> 0, finite) and weight
 *    (finite).  Both sets are copied at create; the caller keeps its arrays.
 *  - Rotations are unit quaternions (w, x, y, z), Hamilton convention; they are
 *    normalised here; a quaternion of norm < 1e-12 or with a non-finite entry
 *    is rejected.  B turns about its own frame origin, then moves by t.
 *  - Translations t = origin + (box / n) * (ix, iy, iz), 0 <= i < n; scores are
 *    stored [rot][iz][iy][ix] (ix fastest) as float, in volume units.
 *  - Device pointers are HIP device memory of the device that was current at
 *    create; all work is enqueued on the stream given at create (NULL = the
 *    null stream) and is asynchronous: synchronise that stream before reading.
 *  - Every call returns CORR_OK or a negative error code; no exception crosses
 *    this boundary.  After an error the context is still valid (or was not
 *    created) and corr_last_error() holds a message.
 *  - Calls on one context must not overlap (one host thread at a time).
 */
#ifndef CORR_H
#define CORR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CORR_OK            0
#define CORR_EINVAL       -1  /* bad argument: value, size, NULL where not allowed */
#define CORR_ENOMEM       -2  /* device or host allocation failed                  */
#define CORR_EHIP         -3  /* a HIP runtime call or kernel launch failed         */
#define CORR_EUNSUPPORTED -4  /* valid but unsupported parameter (grid size, ...)  */

/* flags of corr_grid */
#define CORR_DETERMINISTIC 1u /* bit-reproducible results; accepted for clarity: every
                                 run already is (spreading sums are exact 64-bit
                                 fixed point, independent of scheduling)           */
#define CORR_SC_SCORE      2u /* score the shape complementarity of Sec. 4.2, eq.
                                 eq_score, instead of the overlap: each shape's
                                 defining function f_S becomes its affinity
                                 a_S = f_{S (+) B(0, sc_offset)} - sc_lambda f_S, the
                                 offset of a union of balls being the union of its
                                 balls grown by sc_offset, and the score is
                                 <a_A, a_{(R,t)B}> (the affinity's factor i cancels) */
#define CORR_LIFTED_SCORE  4u /* score slices of the 4D lifted correlation of
                                 Sec. 2.2 (eq. eq_rhoA, eq_L2cone, eq_coneconv) and
                                 Sec. 3.1 (Lemma 2, eq. eq_ORA, eq_convgA): each
                                 ball (x, r) of A lifted to a downward half-cone
                                 {(y, s) : |y - x| <= r - s}, each ball of B to the
                                 r-mirrored upward cone, B moved by the 4D
                                 translation (R, t, h).  The slice at height h is
                                   g_h(R, t) = sum_i sum_j c_i d_j W(|x_i - R y_j - t|; r_i + rho_j - h),
                                 W(d; P) = pi (P^2 - d^2)^2 / 24 for d < P (the 4D
                                 volume of the two cones' intersection), else 0.
                                 Its positive set is the configuration obstacle of
                                 the balls offset by a total of -h (Lemma 2 at
                                 h = 0).  corr_eval gives h = 0; corr_set_offsets
                                 sets other heights.  Not with CORR_SC_SCORE;
                                 corr_spectrum and the queries are not available. */

typedef struct {
    double x, y, z; /* centre                */
    double r;       /* radius, finite, > 0   */
    double w;       /* weight, finite        */
} corr_ball;

typedef struct {
    int32_t n;         /* translations per axis: 16, 32, 64, 128 or 256           */
    double box;        /* period L > 0 of the translation grid; h = box / n       */
    double origin[3];  /* translation at index (0, 0, 0)                          */
    double sigma;      /* oversampling of the spreading grid; 2.0 (0 = default 2) */
    int32_t kb_width;  /* Kaiser-Bessel window width in fine cells: even, 6..12
                          (0 = default 8); 4 is rejected (CORR_EUNSUPPORTED): its
                          window error, ~1e-3, exceeds the 1e-4 tolerance          */
    double tol;        /* tolerance of the radius expansion of the ball transform,
                          relative to the largest ball volume (0 = default 1e-6)   */
    uint32_t flags;    /* CORR_DETERMINISTIC or 0                                  */
    int32_t batch;     /* rotations per pipeline pass, 1..256 (0 = largest that
                          fits a 4 GiB workspace, at most 64)                     */
    double sc_offset;  /* with CORR_SC_SCORE: skin offset r0 >= 0 (length units);
                          otherwise must be 0                                      */
    double sc_lambda;  /* with CORR_SC_SCORE: penalty factor lambda >= 0; otherwise
                          must be 0.  tol is then relative to the volume of the
                          largest grown ball.                                      */
    double lift_range; /* with CORR_LIFTED_SCORE: slice heights h in
                          [-lift_range, min(lift_range, (r_min(A) + r_min(B)) / 2)]
                          are allowed; the radius expansions are planned for
                          them (tol relative to the largest kernel value
                          What(0; r_max(A) + r_max(B) + lift_range)).  Finite,
                          >= 0; otherwise must be 0.                               */
} corr_grid;

typedef struct corr_ctx corr_ctx;

/* Plan of a context, for reporting and for byte models. */
typedef struct {
    int32_t n;          /* translation grid per axis                        */
    int32_t m;          /* spreading grid per axis (sigma * n)              */
    int32_t kb_width;   /* window width                                     */
    int32_t q_a, q_b;   /* radius-expansion components of A and of B        */
    int64_t n_a, n_b;   /* ball counts                                       */
    int32_t batch;      /* rotations processed per pipeline pass            */
    int64_t workspace_bytes; /* device memory held by the context            */
    double beta;        /* Kaiser-Bessel shape parameter                    */
    double radius_err_a, radius_err_b; /* achieved expansion error          */
} corr_info_t;

/*
 * Create a context for shapes A (fixed) and B (rotated).  Validates the input,
 * plans the grids and the radius expansion, copies both ball sets to the
 * device and computes A's spectrum on `hip_stream` (a hipStream_t, or NULL).
 * Either set may be empty: its scores are then identically zero.
 * On success *out owns device memory until corr_destroy.
 */
int corr_create(const corr_ball* A, int64_t nA, const corr_ball* B, int64_t nB,
                const corr_grid* grid, void* hip_stream, corr_ctx** out);

/* Recompute A's spectrum from the device-resident balls of A (the first stage
 * of corr_create, without any host transfer).  Asynchronous: the work is forked
 * from the context's stream onto a private side stream of the library (default
 * priority) with buffers of its own, so that it overlaps the rotated shape's
 * first stages in the next corr_eval; every later call on the context joins it
 * into the context's stream before it reads A's spectrum or the context's
 * device state (corr_eval before its product stage).  Contexts of a batch
 * compute it on the batch's stream. */
int corr_prepare_a(corr_ctx* ctx);

/*
 * Score n_rot rotations of B against A.
 *   quat_wxyz    host array [n_rot][4] (read before return).
 *   scores_dev   device float [n_rot][n][n][n], or NULL to skip the scores.
 *   peak_val_dev device float [n_rot] (largest score of each rotation), or NULL.
 *   peak_idx_dev device int64 [n_rot] (its linear index iz*n*n + iy*n + ix; the
 *                lowest index wins ties), or NULL; must be NULL iff peak_val_dev is.
 * n_rot = 0 is allowed and does nothing.  Asynchronous.
 */
int corr_eval(corr_ctx* ctx, const double* quat_wxyz, int64_t n_rot,
              float* scores_dev, float* peak_val_dev, int64_t* peak_idx_dev);

/*
 * One shape's band-limited spectrum F(k_m) = sum_i c_i Bhat(|k_m|; r_i) exp(-i k_m . R x_i)
 * (Sec. 2.5 eq. eq_rhoPhat weighted by the ball transform) on the half cube of
 * modes: out_dev is device float [n][n][n/2][2] (re, im) indexed
 * [mz][my][mx] with mx = 0 .. n/2-1 and my, mz in FFT order (index i holds mode
 * i for i < n/2, i - n otherwise; index n/2 holds zero).  which = 0 gives A
 * (quat ignored), which = 1 gives B turned by quat_wxyz (host, 4 doubles).
 * Exposes the first three pipeline stages for per-stage checks.  Asynchronous.
 */
int corr_spectrum(corr_ctx* ctx, int32_t which, const double* quat_wxyz, float* out_dev);

int corr_info(const corr_ctx* ctx, corr_info_t* out);

/* Stage ids reported by corr_profile_read. */
#define CORR_STAGE_ROTATE         0  /* a0: turn, place, window weights, sort keys    */
#define CORR_STAGE_BIN            1  /* a0: sorted knot records + live-tile plan      */
#define CORR_STAGE_SPREAD_FFT_X   2  /* a1 + a2: spreading fused with the x pass      */
#define CORR_STAGE_FFT_Y          3  /* a2: forward y pass                            */
#define CORR_STAGE_FFT_Z_SPECTRUM 4  /* a2 z pass + a3, for A or corr_spectrum; with
                                        several slices also B's z sums, once           */
#define CORR_STAGE_FFT_Z_PRODUCT  5  /* a2 z pass + a3 + a4 + inverse z, for B; with
                                        several slices a4 + inverse z per slice        */
#define CORR_STAGE_IFFT_Y         6  /* a5: inverse y pass                            */
#define CORR_STAGE_IFFT_X         7  /* a5: inverse x pass (to real) + block peaks    */
#define CORR_STAGE_PEAK           8  /* a5: per-rotation peak                         */
#define CORR_STAGE_QUERY          9  /* single-configuration query (corr_query)       */
#define CORR_STAGE_GRAPH         10  /* a whole evaluation replayed as one hipGraph
                                        (corr_tuning.graph); its stages are not timed
                                        one by one                                      */
#define CORR_STAGE_RASTER        11  /* the rasterization baseline (corr_raster_eval),
                                        one rotation                                    */
#define CORR_N_STAGES            12

/* Turn per-stage timing on (enable != 0) or off.  While on, every stage launch
 * on the context's stream is bracketed by a pair of HIP events. */
int corr_profile(corr_ctx* ctx, int32_t enable);

/* Wait for the context's stream, then write, per stage id < n_stages, the
 * summed device time in milliseconds (ms) and the number of launches timed
 * since the last read; clears the record. */
int corr_profile_read(corr_ctx* ctx, double* ms, int64_t* launches, int32_t n_stages);

/*
 * Time-critical score of single configurations (Sec. 4.1, eq. eq_single): for
 * B turned by quat_wxyz (host, 4 doubles), the band-limited score at n_t
 * arbitrary translations t_host (host double [n_t][3], any position, not only
 * grid points), as the Parseval sum
 *   s(t) = (1/L^3) sum_m F_A(k_m) conj(F_RB(k_m)) exp(i k_m . t)
 * over the modes with |m|^2 <= mode_radius2 and |m_d| < n/2: a ball of modes
 * grown from the dominant low modes, trading accuracy for time.  A radius of
 * 3 (n/2 - 1)^2 or more keeps every mode, which at grid points is the score of
 * corr_eval.  F_A is the fixed shape's prepared spectrum; F_RB is evaluated at
 * the kept modes directly from B's knots (no spreading grid).  Writes out_dev
 * (device float [n_t]) asynchronously on the context's stream; if n_modes is
 * not NULL it receives the number of modes summed (counting m and -m).  A
 * score kind set at create (CORR_SC_SCORE) applies here too.
 */
int corr_query(corr_ctx* ctx, const double* quat_wxyz, const double* t_host, int64_t n_t, int32_t mode_radius2,
               float* out_dev, int64_t* n_modes);

/*
 * corr_query for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same arguments,
 * kernels and summation order as corr_query, hence bitwise its results, but no
 * device, pinned or host heap allocation.  Its device buffers come from one
 * static device array of 32 MiB per GPU (held by each GPU the library runs on
 * until the process ends), shared by every call on that GPU: calls on one GPU
 * must not overlap (they would race on it), whatever their contexts and
 * streams.  The mode list, rotation and translations are copied into it from
 * the caller's host memory (pageable copies on the context's stream; the
 * caller's arrays may be reused on return).  Limits: at most 65536 half-space
 * modes (mode_radius2 up to about 630 on grids with n >= 64), and all buffers
 * of the call within the 32 MiB (about 8 n_modes x ceil(n_B / 256) + 28 n_t
 * bytes); a larger request fails with CORR_EUNSUPPORTED before any device
 * work.  Other errors as corr_query.
 */
int corr_query_noalloc(corr_ctx* ctx, const double* quat_wxyz, const double* t_host, int64_t n_t,
                       int32_t mode_radius2, float* out_dev, int64_t* n_modes);

/*
 * The uniform-rasterization baseline (Sec. 5.2 and Sec. 6.2: the grid method
 * the nonequispaced route is compared with).  Both unions are sampled on the
 * context's translation grid: A at origin + h u and B, turned by rotation r, at
 * h v (u, v in [0, n)^3, v read as the signed index of FFT order), a sample
 * being 1 when it lies in some ball (|p - c|^2 <= r^2, FP64).  The two sample
 * grids are correlated by FFT (FP64: one packed forward transform, the
 * pointwise product, one inverse transform), so that
 *   counts_dev[r][tz][ty][tx] = sum_u a(u) b(u - t)   (periodic indices)
 * is the exact number of samples where A meets B moved by origin + h t; h^3
 * times it estimates vol(A & (R B + t)), the overlap of the two unions (a ball
 * overlap inside a shape counts once).  counts_dev: device int32
 * [n_rot][n][n][n]; quat_wxyz host [n_rot][4].  Independent of the score kind
 * set at create.  Works on buffers grown on demand (n^3 x 16 bytes).
 * Asynchronous.
 */
int corr_raster_eval(corr_ctx* ctx, const double* quat_wxyz, int64_t n_rot, int32_t* counts_dev);

/* ---- configuration obstacles and offset slices --------------------------- */

#define CORR_MAX_SLICES 16

/*
 * Offset obstacles (Sec. 3.1: the slices of the lifted obstacle away from
 * r = 0 are the obstacles of the primitives offset by a total r).  Sets the
 * radius offsets delta_k used by corr_eval_slices: slice k scores
 *     s_k(R, t) = < f_{A_k}, f_{(R,t)B} >,  A_k = A with every radius r_i + delta_k,
 * whose positive set is the translational configuration obstacle grown by
 * delta_k (shrunk for delta_k < 0): the translations where some pair of balls
 * comes closer than r_i + rho_j + delta_k.
 *   offsets    host double [n_offsets], copied; each finite with
 *              r_i + delta_k > 0 for every ball of A.
 *   n_offsets  0 .. CORR_MAX_SLICES; 0 clears the list (then corr_eval_slices
 *              has one slice, the context's own score).
 * Plans each offset shape and computes its spectrum on the context's stream;
 * returns after that work is done.  The B side is shared: per rotation, B is
 * spread and transformed once for all slices.
 * Errors: CORR_EINVAL (bad value or count), CORR_EUNSUPPORTED (with
 * CORR_SC_SCORE, whose kernel already offsets the balls), CORR_ENOMEM, CORR_EHIP.
 * After an error the previous offsets stay in force.
 * With CORR_LIFTED_SCORE the values are slice heights h_k of the lifted
 * correlation instead (slice k scores g_{h_k}, whose positive set is the
 * obstacle offset by -h_k), each within the range planned at create
 * (corr_grid.lift_range); A's component spectra are shared by all heights.
 */
int corr_set_offsets(corr_ctx* ctx, const double* offsets, int32_t n_offsets);

/* Outputs of corr_eval_slices; every pointer is device memory or NULL (not
 * produced).  S = number of slices (offsets set, or 1), R = n_rot. */
typedef struct {
    float* scores;            /* float [S][R][n][n][n]                                  */
    float* peak_val;          /* float [S][R]: largest score of each rotation            */
    int64_t* peak_idx;        /* int64 [S][R]: its linear index (lowest wins ties);
                                 set iff peak_val is                                      */
    uint32_t* obstacle;       /* uint32 [S][R][n^3 / 32]: bit b of word w is set iff the
                                 score at linear index 32 w + b exceeds threshold: the
                                 translational configuration obstacle of Sec. 3.1
                                 eq. eq_obs (threshold 0) as a bit mask                   */
    int64_t* obstacle_count;  /* int64 [S][R]: translations in the obstacle               */
    float threshold;          /* finite, in score (volume) units; the comparison is
                                 made on the float score, exactly as stored in scores     */
} corr_slices_out;

/*
 * Score n_rot rotations of B (host quat_wxyz [n_rot][4]) against every slice
 * of corr_set_offsets (or against A alone if none are set) and write the
 * requested outputs.  The obstacle bits are the configuration-obstacle
 * predicate of the band-limited score; with a threshold of 0 the band limit's
 * ringing also marks points near the obstacle, so a small positive threshold
 * is the usual choice.  Asynchronous.
 */
int corr_eval_slices(corr_ctx* ctx, const double* quat_wxyz, int64_t n_rot, const corr_slices_out* out);

/* Occupancy of the last spreading pass run by ctx (the rotations of the last
 * batch of corr_eval, or one shape for corr_prepare_a / corr_spectrum).  The
 * spreading grid of a rotation is cut into m z rows x (m / tile_rows) tiles of
 * tile_rows y rows; a tile or z row is live when some knot's window reaches
 * it.  Only live tiles are spread and transformed, and the later passes read
 * only live rows.  Synchronises the context's stream.  With a batch, valid
 * until any pair of the batch runs another pass. */
typedef struct {
    int32_t rotations;   /* rotations in the pass                            */
    int32_t q;           /* radius-expansion components of the shape spread  */
    int32_t tile_rows;   /* y rows per tile                                  */
    int32_t m;           /* spreading grid per axis                          */
    int64_t knots;       /* balls of the shape spread                        */
    int64_t tiles;       /* rotations * m * (m / tile_rows)                  */
    int64_t live_tiles;  /* tiles that some knot's window reaches            */
    int64_t live_rows;   /* z rows (over all rotations) with a live tile     */
} corr_pass_t;

int corr_pass_info(corr_ctx* ctx, corr_pass_t* out);

/* Work of the spreading launches (stage CORR_STAGE_SPREAD_FFT_X) since the
 * last read, which clears it: out[0] bytes of kept x modes written (live tiles
 * only, counted by the kernel on the device), out[1] bytes of the sorted knot
 * records of the passes (cell, 3 w window weights and q component weights per
 * knot and rotation), out[2] launches; A's side-stream passes included.
 * These are the algorithmic bytes of the spreading kernel: each record read
 * once, each kept mode written once.  Counted in graph replays too.
 * Synchronises the context's stream.  out: host int64 [3]. */
int corr_spread_work(corr_ctx* ctx, int64_t* out);

/* ---- launch shapes, autotuning and graph replay --------------------------- */

/*
 * How a context cuts its pipeline into launches.  No setting changes the
 * arithmetic or its order, so every tuning gives bitwise the same outputs; only
 * the time differs.  A new context starts from the defaults (the slot count of
 * corr_grid.batch, two spreading workgroups per CU, each pass's default width,
 * graph off).
 */
typedef struct {
    int32_t slots;       /* rotations per pipeline pass, 1..256; changing it reallocates
                            the workspace (after the stream has drained)               */
    int32_t spread_wgs;  /* persistent workgroups of the spreading pass, 1 .. 2 x CUs   */
    int32_t cols_y;      /* columns per forward-y workgroup                              */
    int32_t cols_z;      /* columns per z-pass workgroup                                 */
    int32_t cols_iy;     /* columns per inverse-y (and slice-product) workgroup          */
    int32_t pairs_ix;    /* line pairs per inverse-x workgroup                           */
    int32_t graph;       /* 1: corr_eval and corr_eval_slices capture all launches of a
                            call (every batch of rotations) into a hipGraph on a private
                            stream and replay it with one hipGraphLaunch on the
                            context's stream.  The graph is kept and replayed while the
                            call's n_rot, output pointers and threshold, the slices and
                            the tuning stay the same; otherwise it is captured again.
                            The rotations are copied to a device array first (one
                            host-to-device copy per call).  0: launch by launch.     */
    int32_t bin_group;   /* y cells per sort key of the spreading pass's binning (keys
                            are z-cell x y-group): the grid's default, half or twice
                            it, as corr_tuning_choices(pass 4) lists                 */
    int32_t tile_rows;   /* y rows of a spreading tile (one z row each): the grid's
                            default or half of it, as corr_tuning_choices(pass 5)
                            lists                                                    */
} corr_tuning;

/* The context's current tuning. */
int corr_get_tuning(const corr_ctx* ctx, corr_tuning* out);

/* Set every field (start from corr_get_tuning).  The widths must be among
 * corr_tuning_choices.  Errors: CORR_EINVAL (a value outside its choices),
 * CORR_ENOMEM / CORR_EHIP (workspace); the old tuning then stays in force
 * unless the workspace was lost. */
int corr_set_tuning(corr_ctx* ctx, const corr_tuning* tuning);

/* The widths allowed for column pass `pass` (0 cols_y, 1 cols_z, 2 cols_iy,
 * 3 pairs_ix) on this context's grid: the default first, then half and twice
 * it where the pass's shape allows; pass 4: the bin_group values (the default
 * first, then half and twice it where the grid's key count stays within
 * 1024 .. 32768); pass 5: the tile_rows values (the default, then half of it).
 * out3 receives *count (1..3) values. */
int corr_tuning_choices(const corr_ctx* ctx, int32_t pass, int32_t* out3, int32_t* count);

/* flags of corr_autotune */
#define CORR_TUNE_WITH_A 1u  /* time corr_prepare_a + corr_eval as one unit (the fixed
                                shape's spectrum is recomputed with every
                                evaluation), not corr_eval alone                  */

/*
 * Autotuner.  Evaluates these rotations (arguments as for corr_eval) under
 * candidate tunings and keeps the fastest: coordinate descent over slots
 * (powers of two up to n_rot, workspace <= 8 GiB), spread_wgs (one, one and a
 * half or two per CU), the four column widths, the bin group and the tile
 * height, each candidate timed by HIP
 * events as the least of `reps` (1..100) runs after an untimed one.  A run is
 * corr_eval, or with CORR_TUNE_WITH_A corr_prepare_a + corr_eval.  The graph
 * setting is kept as it is.  Synchronous; the outputs hold the last
 * evaluation's results, which equal corr_eval's under any tuning.  *out (may
 * be NULL) receives the tuning kept.
 */
int corr_autotune(corr_ctx* ctx, const double* quat_wxyz, int64_t n_rot, float* scores_dev, float* peak_val_dev,
                  int64_t* peak_idx_dev, int32_t reps, uint32_t flags, corr_tuning* out);

/* ---- uneven batches of pairs --------------------------------------------- */

/* One shape pair with its own translation grid (grid.batch is ignored). */
typedef struct {
    const corr_ball* A;
    int64_t nA;
    const corr_ball* B;
    int64_t nB;
    corr_grid grid;
} corr_pair;

typedef struct corr_batch corr_batch;

/*
 * Plan every pair (ball counts and grid sizes may all differ) and share one
 * device workspace among them.  Rotations per pass (corr_batch_info's batch):
 *   slots = 0   per pair, the most (at most 64) whose buffers fit 8 GiB for that
 *               pair; each workspace buffer is sized for the pair needing most
 *               of it, so pairs on small grids run many rotations per pass;
 *   slots > 0   `slots` for the pair needing most, and as many as fit in the
 *               same buffers for the others (at most 256).
 * Computes every A spectrum.  Pair p is validated like corr_create; its errors
 * name the pair.
 */
int corr_batch_create(const corr_pair* pairs, int32_t n_pairs, int32_t slots, void* hip_stream,
                      corr_batch** out);

/*
 * Score rotation r = rot_offsets[p] .. rot_offsets[p+1]-1 (host quaternions
 * quat_wxyz[r]) of pair p, for every p.  rot_offsets: host int64 [n_pairs + 1],
 * starting at 0, non-decreasing.  scores_dev (or NULL): pair p's
 * [rotations][n_p][n_p][n_p] block starts at float offset score_offsets[p]
 * (host int64 [n_pairs]), or, with score_offsets NULL, the blocks are packed in
 * pair order.  peak_val_dev / peak_idx_dev (device, [rot_offsets[n_pairs]],
 * both or neither): per-rotation peaks as in corr_eval.  Asynchronous.
 */
int corr_batch_eval(corr_batch* b, const double* quat_wxyz, const int64_t* rot_offsets, float* scores_dev,
                    const int64_t* score_offsets, float* peak_val_dev, int64_t* peak_idx_dev);

/* enable = 1: corr_batch_eval captures all pairs' launches of a call into one
 * hipGraph and replays it with one hipGraphLaunch while the call's rotation
 * offsets, score offsets and output pointers stay the same (see
 * corr_tuning.graph); 0: launch by launch (the default). */
int corr_batch_set_graph(corr_batch* b, int32_t enable);

int corr_batch_info(const corr_batch* b, int32_t pair, corr_info_t* out);

/*
 * Autotuner of a batch: runs corr_batch_eval (these arguments) under candidate
 * launch shapes and keeps the fastest, by coordinate descent: spread_wgs (one,
 * one and a half or two per CU, for every pair), then, for each grid size of
 * the batch in turn (largest first, applied to the pairs on that grid), each
 * column pass's width, the bin group and the tile height, each by rank among
 * each pair's own choices (0 the pair's default, 1 and 2 the others of
 * corr_tuning_choices where its grid has them).  Rotations per pass stay as
 * planned at create.  Each candidate is timed by HIP events as the least of
 * `reps` (1..100) runs after an untimed one.  No tuning changes a bit of the
 * outputs, which hold the last evaluation.  Synchronous.  out7 (host int32
 * [7], or NULL): spread_wgs, and the four column ranks, the bin-group rank
 * and the tile-height rank kept for the batch's largest grid.  After an error
 * the pairs' previous tunings are restored.
 */
int corr_batch_autotune(corr_batch* b, const double* quat_wxyz, const int64_t* rot_offsets, float* scores_dev,
                        const int64_t* score_offsets, float* peak_val_dev, int64_t* peak_idx_dev, int32_t reps,
                        int32_t* out7);

/* corr_profile / corr_profile_read over every pair of the batch (the read
 * sums the pairs' stage times and launch counts), and corr_spread_work of the
 * batch's shared workspace. */
int corr_batch_profile(corr_batch* b, int32_t enable);
int corr_batch_profile_read(corr_batch* b, double* ms, int64_t* launches, int32_t n_stages);
int corr_batch_spread_work(corr_batch* b, int64_t* out);
int corr_batch_destroy(corr_batch* b);
const char* corr_batch_last_error(const corr_batch* b);

/* Free the context and its device memory (waits for its stream).  NULL is a no-op. */
int corr_destroy(corr_ctx* ctx);

/* Message of the last failed call on ctx; with ctx = NULL, the last failure of
 * a call without a context on this thread (e.g. corr_create).  Never NULL. */
const char* corr_last_error(const corr_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* CORR_H */

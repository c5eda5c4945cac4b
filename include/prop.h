/*
 * prop.h -- C ABI of the rotation-proposal network in libcorr.so.
 *
 * A small MLP learns, for a pair of ball-union shapes, the peak correlation
 * score reached at a rotation, so that a rotation search runs the full
 * correlation (corr.h) only on the candidates the network ranks highest, with
 * exhaustive evaluation as the fallback and as the judge of its recall.  The
 * correlation whose peaks it learns is the score of Behandish & Ilies (CAD
 * 2016), Sec. 3.1 eq. eq_relg_0, evaluated by the Fourier route of Sec. 3.2.
 *
 * Network: layers 160 -> 256 -> 256 -> 256 -> 1 with ReLU between.  Inputs
 * (155 used, zero-padded to 160):
 *   x[0..8]     the rotation matrix R(q) of the quaternion, row-major (the same
 *               for q and -q, and continuous over all rotations, which a
 *               canonical quaternion with w >= 0 is not across w = 0);
 *   x[9..17]    sin(pi R_e) and x[18..26] cos(pi R_e) of each entry (a fixed
 *               Fourier feature map of the rotation);
 *   x[27..90]   64 * descriptor of A, x[91..154] 64 * descriptor of B (scaled
 *               by the bin count so that an entry is 1 on average).
 * A descriptor is the histogram of ball volume (weight * r^3) over the
 * distance of each centre from the volume-weighted centroid, 64 bins of width
 * 1/64 on [0, 1] (farther centres in the last bin), normalised to sum 1.
 *
 * Arithmetic: the layer products run on the matrix cores with bfloat16 weights
 * and bfloat16 layer inputs, accumulating in FP32 (forward and backward);
 * biases, losses, gradients' reductions and the Adam state are FP32, and Adam
 * updates FP32 master weights from which the bfloat16 copies are re-rounded.
 * Loss: mean squared error.
 *
 * Conventions as in corr.h: device pointers belong to the device current at
 * create, work is enqueued on the stream given at create and is asynchronous
 * unless stated; negative return codes (CORR_E*) with prop_last_error().
 */
#ifndef PROP_H
#define PROP_H

#include <stdint.h>

#include "corr.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PROP_IN      160  /* padded input width                  */
#define PROP_HIDDEN  256  /* hidden width                        */
#define PROP_BINS     64  /* descriptor bins                     */
#define PROP_NPARAMS (160 * 256 + 256 + 2 * (256 * 256 + 256) + 256 + 1)

typedef struct prop_ctx prop_ctx;

/* New network with He-uniform weights drawn from `seed` and zero biases.
 * batch: training mini-batch size, 64..8192, a multiple of 64. */
int prop_create(int32_t batch, uint64_t seed, void* hip_stream, prop_ctx** out);

/* Descriptor of a ball set (host corr_ball[n], n >= 1; finite centres, radii
 * > 0 and weights > 0, else CORR_EINVAL) into desc_dev[64] (device float): the
 * histogram of the volumes w r^3 over the centres' distance from the
 * volume-weighted centroid, normalised to sum 1. */
int prop_descriptor(prop_ctx* p, const corr_ball* balls, int64_t n, float* desc_dev);

/* Network inputs X_dev[n][160] (device float, layout above) for n quaternions
 * (host double [n][4], any non-zero norm) and two device descriptors. */
int prop_features(prop_ctx* p, const double* quat_wxyz, int64_t n, const float* desc_a_dev,
                  const float* desc_b_dev, float* X_dev);

/* Train on n samples (X_dev[n][160], y_dev[n], device float) for `epochs`
 * passes of shuffled mini-batches (the last partial batch of each pass is
 * dropped; n >= batch required) with Adam at learning rate lr.  If loss_host is
 * not NULL it receives the mean training loss of each epoch (host float
 * [epochs]); that read synchronises the stream. */
int prop_train(prop_ctx* p, const float* X_dev, const float* y_dev, int64_t n, int32_t epochs, float lr,
               float* loss_host);

/* Predicted peak score of n inputs into y_dev[n] (device float). */
int prop_predict(prop_ctx* p, const float* X_dev, int64_t n, float* y_dev);

/* Indices of the k inputs with the highest predicted score (ties: lower index
 * first), in decreasing order of score, into idx_dev[k] (device int64).
 * 1 <= k <= n <= 8192 (one workgroup sorts the scores in LDS); larger n
 * returns CORR_EUNSUPPORTED. */
int prop_rank(prop_ctx* p, const float* X_dev, int64_t n, int32_t k, int64_t* idx_dev);

/* Mean-squared-error gradient of one batch of n <= batch samples without an
 * update: grads_host receives PROP_NPARAMS floats in the parameter order of
 * prop_get_params.  Synchronises the stream. */
int prop_gradient(prop_ctx* p, const float* X_dev, const float* y_dev, int64_t n, float* grads_host);

/* FP32 master parameters, PROP_NPARAMS floats: W1 [160][256], b1 [256],
 * W2 [256][256], b2, W3 [256][256], b3, W4 [256], b4 [1] (W[l] is [in][out]).
 * get synchronises the stream; set also resets the Adam state. */
int prop_get_params(prop_ctx* p, float* host_out);
int prop_set_params(prop_ctx* p, const float* host_in);

int prop_destroy(prop_ctx* p);

/* Message of the last failed call on p (or, with p = NULL, of this thread). */
const char* prop_last_error(const prop_ctx* p);

#ifdef __cplusplus
}
#endif

#endif /* PROP_H */

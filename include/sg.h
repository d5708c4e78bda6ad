/*
 * sg.h -- C ABI of the CNN surrogate that warm-starts steady-state runs of the
 * lattice Boltzmann solver (lb.h).  Project addition: the paper defines no
 * learned component; the network maps the parameters of a double-diffusive
 * cavity (Sec. 3.2: Ra, Le, Nc, Sr = S_TC, Df = D_CT) plus the grid
 * coordinates to the steady fields (u, v, T, C), and the LB iteration remains
 * what decides its error.
 *
 * Network (fixed): six 3x3 convolutions, zero padding, channels-last
 *   15 -> 64 -> 128 -> 64 -> 64 -> 64 -> 4, SiLU after each hidden layer.
 * Input features per pixel: the 5 normalised parameters, the cell-centre
 * coordinates xc = (i + 1/2)/W, yc = (j + 1/2)/H and sin/cos of pi xc, 2 pi xc,
 * pi yc, 2 pi yc.  Weights and activations are stored in bfloat16, products
 * accumulate in FP32 on the gfx950 matrix cores; master weights, the loss
 * (mean squared error over the 4 outputs) and Adam run in FP32.
 *
 * Packed parameter vector (FP32), layer by layer: w[co][tap][ci] with
 * tap = (dy + 1) * 3 + (dx + 1) (input pixel (y + dy, x + dx)), over the padded
 * channel counts of sg_layer_info, then b[co].  Padded entries must be 0 and
 * stay 0.
 *
 * Device arrays: params [n][5] FP32 (normalised), fields [n][4][H][W] FP32
 * (u, v, T, C).  Ownership, errors and streams as in lb.h.
 */
#ifndef LBCDF_SG_H
#define LBCDF_SG_H

#include <stddef.h>
#include <stdint.h>

#include "lb.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SG_LAYERS 6
#define SG_IN_PARAMS 5
#define SG_OUTPUTS 4

typedef struct sg_config {
    int32_t batch;        /* samples per training step / largest prediction batch */
    int32_t height, width;/* grid; width a multiple of 64 */
    int32_t reserved;     /* must be 0 */
    float lr, beta1, beta2, eps; /* Adam */
} sg_config;

typedef struct sg_handle sg_handle;

/* Real and padded channel counts of layer l (0..SG_LAYERS-1). */
lb_status sg_layer_info(int32_t layer, int32_t* cin, int32_t* cout, int32_t* cin_pad, int32_t* cout_pad);

/* Length of the packed parameter vector (padded) and number of real parameters. */
lb_status sg_param_count(int64_t* packed, int64_t* real);

lb_status sg_workspace_bytes(const sg_config* cfg, size_t* bytes);
lb_status sg_create(const sg_config* cfg, void* dev_workspace, size_t workspace_bytes, void* hip_stream,
                    sg_handle** out);

/* Host copies of the FP32 master weights (packed layout); set also resets Adam. */
lb_status sg_set_weights(sg_handle* h, const float* host_packed);
lb_status sg_get_weights(sg_handle* h, float* host_packed);

/* Loss and gradients of one batch without updating: samples host_idx[0..batch)
 * of the device arrays.  loss_out (host) and grads_out (host, packed) may be NULL. */
lb_status sg_gradients(sg_handle* h, const float* d_params, const float* d_fields, const int32_t* host_idx,
                       float* loss_out, float* grads_out);

/* One Adam step on one batch (as sg_gradients, then the update). */
lb_status sg_train_step(sg_handle* h, const float* d_params, const float* d_fields, const int32_t* host_idx,
                        float* loss_out);

/* Epochs over n samples in seeded shuffled order (full batches only);
 * losses_out[epoch] = mean batch loss.  Synchronises. */
lb_status sg_train_epochs(sg_handle* h, const float* d_params, const float* d_fields, int32_t n, int32_t epochs,
                          uint64_t seed, float* losses_out);

/* Prediction for n samples (any n; processed in chunks of the batch size):
 * d_out [n][4][H][W] FP32 on the device.  Asynchronous. */
lb_status sg_predict(sg_handle* h, const float* d_params, int32_t n, float* d_out);

/* Pre-activations z of layer l from the last forward pass, host [batch][H][W][cout_pad]. */
lb_status sg_layer_output(sg_handle* h, int32_t layer, float* host_out);

/* Input of layer l (bfloat16 values widened to FP32) from the last forward
 * pass, host [batch][H][W][cin_pad]. */
lb_status sg_layer_input(sg_handle* h, int32_t layer, float* host_out);

/* One 3x3 convolution of layer l, run by the same kernels and launch shapes as
 * the training pass, on caller-owned device tensors of nb <= batch samples
 * (channels-last, padded channel counts of sg_layer_info; bf16 arrays are
 * raw bfloat16 words).  Uses the handle's current bfloat16 weights.
 *   mode 0 (forward): z = b_l + sum_{tap, ci} w_l[co][tap][ci] x[p + off(tap)][ci]
 *     with x = d_in [nb][H][W][cin_pad]; d_z [nb][H][W][cout_pad] FP32 receives z
 *     (may be NULL), d_out [nb][H][W][cout_pad] bf16 receives bf16(SiLU(z)) for
 *     hidden layers and bf16(z) for the last; d_zprev is ignored.
 *   mode 1 (data gradient, l >= 1): with g = d_in [nb][H][W][cout_pad] (dL/dz of
 *     layer l), d_out [nb][H][W][cin_pad] bf16 receives
 *     bf16(SiLU'(zprev) sum_{tap, co} w_l[co][tap][ci] g[p - off(tap)][co]),
 *     the gradient with respect to the pre-activation of layer l - 1;
 *     d_zprev [nb][H][W][cin_pad] FP32 is that pre-activation; d_z is ignored.
 * Asynchronous on the handle's stream. */
lb_status sg_conv(sg_handle* h, int32_t layer, int32_t mode, int32_t nb, const void* d_in, const float* d_zprev,
                  float* d_z, void* d_out);

/* Weight and bias gradients of layer l for nb <= batch samples, by the
 * kernels of the training pass: d_dw [cout_pad][9][cin_pad] FP32 receives
 * sum_p g[p][co] x[p + off(tap)][ci] and d_db [cout_pad] FP32 sum_p g[p][co],
 * with g = d_g [nb][H][W][cout_pad] and x = d_x [nb][H][W][cin_pad] bf16
 * device tensors.  Both sums run in a fixed order (bitwise reproducible).
 * Uses the handle's reduction scratch.  Asynchronous on the handle's stream. */
lb_status sg_weight_grad(sg_handle* h, int32_t layer, int32_t nb, const void* d_g, const void* d_x, float* d_dw,
                         float* d_db);

/* Separable [1 2 1]/4 x [1 2 1]/4 filter of `planes` device planes of
 * height x width (edge values replicated), d_in -> d_out (not in place),
 * asynchronous on hip_stream.  Applied to predictions before a warm start: it
 * removes the grid-scale (Nyquist) content that the lattice Boltzmann
 * iteration damps very slowly. */
lb_status sg_smooth(const float* d_in, float* d_out, int32_t planes, int32_t height, int32_t width,
                    void* hip_stream);

/* In place on `count` device field sets [count][4][height][width] (u, v, T, C):
 * u -= <u (-1)^x> (-1)^x and v -= <v (-1)^y> (-1)^y, the means taken over
 * the whole plane (FP64 accumulation, deterministic).  Asynchronous on
 * hip_stream.
 * Why: with bounce-back walls (or periodic axes of even length) the D2Q9
 * update conserves the staggered momenta sum (-1)^y j_y and sum (-1)^x j_x up
 * to a sign flip per step, because the collision conserves momentum (the
 * force of Eq. force only adds F) and every population that carries c_y moves
 * to a row of the other parity or is reflected with c_y reversed.  A warm
 * start whose velocity has non-zero staggered sums therefore keeps an
 * undamped period-2 oscillation; with them removed the initial state sits on
 * the fixed point of that recurrence (the fluid is initialised at momentum
 * u0 - F/2, see lb_init). */
lb_status sg_destagger(float* d_fields, int32_t count, int32_t height, int32_t width, void* hip_stream);

lb_status sg_free(sg_handle* h);

/* Thread-local text of the last surrogate error. */
const char* sg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBCDF_SG_H */

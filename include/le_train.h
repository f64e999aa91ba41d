/*
 * le_train.h -- training and checking entry points of the learned
 * coarse-step corrector (companion of le.h; same conventions and error
 * codes).  These take device pointers and expose the network's pieces for
 * its training driver and its tests; the time-step contract of le.h does not
 * need them.
 */
#ifndef LE_TRAIN_H
#define LE_TRAIN_H

#include <stdint.h>

#include "le.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Training the corrector network on the GPU (BF16 matrix-core kernels, FP32
 * accumulation and master weights, Adam).  Pointers named *_dev are device
 * memory (e.g. torch tensors); planes are [channel][H][W] FP32 with channel 0
 * = phi and 1 = omega; batches stack planes: [B][2][H][W].  H, W: powers of
 * two >= 16 with H*W a multiple of 256.  stream: hipStream_t or NULL.
 *
 * le_cnn_grad: loss = mean over the batch, channels and pixels of (r - t)^2
 *   with r the network's output on x, t the target residual; its gradient
 *   replaces the stored one (and is copied to grad_host when non-NULL).
 * le_cnn_adam: one Adam step with the stored gradient.
 * le_cnn_layer_fwd / le_cnn_layer_bwd (layer 0..3) run one convolution on
 *   pixel-major BF16 inputs a_in_dev [H*W][Cin] (bit patterns): forward gives
 *   the FP32 pre-activation [H*W][Cout] (and BF16 SiLU output for layers
 *   0..2); backward takes dz_dev [H*W][Cout] FP32 and gives the weight and
 *   bias gradient dw_dev (that layer's slice of the weight vector) and, for
 *   layers 1..3 when dzprev_dev is given, the input gradient times silu'(zprev)
 *   (zprev_dev NULL: the plain input gradient).
 * le_cnn_mfma_probe: one 32x32x16 BF16 matrix product c = a b on host arrays
 *   (row-major a 32x16, b 16x32 BF16 bit patterns, c 32x32 FP32): a check of
 *   the matrix-core operand layout the convolution kernels assume.
 */
typedef struct le_cnn le_cnn;
int le_cnn_nparams(void);
int le_cnn_create(int32_t H, int32_t W, le_cnn** out);
void le_cnn_destroy(le_cnn* c);  /* NULL-safe */
int le_cnn_set_params(le_cnn* c, const float* params, int32_t n, const float* scales);
int le_cnn_get_params(le_cnn* c, float* params, int32_t n);
int le_cnn_forward(le_cnn* c, const float* x_dev, float* r_dev, void* stream);
int le_cnn_grad(le_cnn* c, const float* x_dev, const float* t_dev, int32_t batch, double* loss,
                float* grad_host, void* stream);
int le_cnn_adam(le_cnn* c, float lr, float beta1, float beta2, float eps, void* stream);
int le_cnn_layer_fwd(le_cnn* c, int32_t layer, const uint16_t* a_in_dev, float* z_out_dev,
                     uint16_t* a_out_dev, void* stream);
int le_cnn_layer_bwd(le_cnn* c, int32_t layer, const float* dz_dev, const uint16_t* a_in_dev,
                     const float* zprev_dev, float* dzprev_dev, float* dw_dev, void* stream);
int le_cnn_mfma_probe(const uint16_t* a, const uint16_t* b, float* c);

#ifdef __cplusplus
}
#endif

#endif /* LE_TRAIN_H */

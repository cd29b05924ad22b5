/* convlearn.h - the learned split network of libconvreal: a 3 -> 64 -> 64 -> 2 perceptron
 * (tanh hidden layers, linear output) that maps (log Nside, log FWHM, log target error), normalised,
 * to a normalised split (theta_cut, l_cut), trained on the device by the library's own forward,
 * back-propagation and Adam kernels (FP32 storage and products, FP64 sums over samples).
 *
 * The network stands beside the paper's split search (Estimating Errors section and the discussion
 * of Table 1): the scan evaluates the error model for many (theta_cut, l_cut) pairs, the network
 * predicts the pair in one forward pass, and the error model judges the prediction.
 *
 * Parameter vector (4546 floats, row-major): W1 [64 x 3], b1 [64], W2 [64 x 64], b2 [64],
 * W3 [2 x 64], b3 [2]. Loss: L = (1 / 2n) sum_s sum_o (y_so - t_so)^2.
 *
 * Device pointers: x [n][3], t [n][2], y [n][2], grad [4546], loss [1], loss_hist [steps], all FP32,
 * caller-owned device memory (for instance torch tensors); host pointers where stated. Calls are
 * asynchronous on `stream` (a hipStream_t, NULL = the default stream) except set/get_params, which
 * synchronise. Return CONV_REAL_OK or a negative CONV_REAL_E* code (convreal.h).
 */
#ifndef CONVLEARN_H
#define CONVLEARN_H

#include "convreal.h"

#ifdef __cplusplus
extern "C" {
#endif

#define CONV_MLP_IN 3
#define CONV_MLP_HIDDEN 64
#define CONV_MLP_OUT 2
#define CONV_MLP_NPARAMS 4546
#define CONV_MLP_MAX_BATCH 1048576

typedef struct conv_mlp conv_mlp;

/* Adam (Kingma & Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
 * p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
typedef struct conv_adam {
  float lr;
  float beta1;
  float beta2;
  float eps;
} conv_adam;

/* Allocates parameters (zero), Adam moments and activation buffers for batches of up to
 * max_batch samples (1 <= max_batch <= CONV_MLP_MAX_BATCH) on the current device. */
int conv_mlp_create(conv_mlp** m, int max_batch);

/* Frees everything; NULL is accepted. */
int conv_mlp_destroy(conv_mlp* m);

/* Copies CONV_MLP_NPARAMS floats from host memory into the network and resets the Adam state
 * (moments and step count). Non-finite values are rejected. Synchronous. */
int conv_mlp_set_params(conv_mlp* m, const float* host_params);

/* Copies the parameters to host memory. Synchronous (waits for the device). */
int conv_mlp_get_params(conv_mlp* m, float* host_params);

/* y = network(x) for n samples (1 <= n <= max_batch). */
int conv_mlp_forward(conv_mlp* m, const float* x, int n, float* y, void* stream);

/* Loss and its gradient with respect to every parameter at the current parameters, for the
 * batch (x, t) of n samples; grad and loss are device pointers. Parameters are unchanged. */
int conv_mlp_gradient(conv_mlp* m, const float* x, const float* t, int n, float* grad, float* loss,
                      void* stream);

/* `steps` full-batch Adam steps on (x, t) (n samples); loss_hist (device, may be NULL) receives the
 * loss before each step. The Adam step count continues across calls until set_params. */
int conv_mlp_train(conv_mlp* m, const float* x, const float* t, int n, int steps, const conv_adam* opt,
                   float* loss_hist, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CONVLEARN_H */

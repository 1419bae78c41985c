/* The surrogate network of the propagation library: a multilayer perceptron
 * that maps (bath parameters, system parameters, time) to rho(t), trained on
 * trajectories of the batched propagation (quapi_create_batch) and checked
 * against it.  The paper does not contain it; it serves parameter scans where
 * a trained network answers in place of the method, which stays the fallback
 * and the judge of its error.
 *
 * Architecture: n_in -> width -> ... -> width -> n_out, depth hidden layers
 * with the exact GELU activation x/2 (1 + erf(x/sqrt 2)), a linear output
 * layer.  Loss: the mean over batch x n_out of (y - target)^2.  Optimiser:
 * Adam (Kingma & Ba 2015).  The matrix products run on the bf16 matrix cores
 * with FP32 accumulation (layer inputs, weights and back-propagated gradients
 * rounded to bf16 as they enter a product); an input layer of at most 16
 * inputs runs in FP32, and everything else is FP32.
 *
 * Parameters, flat FP32, for each layer l = 0 .. depth: W_l [fan_in][fan_out]
 * row-major, then b_l [fan_out].
 *
 * Device pointers: x [batch][n_in], y and target [batch][n_out], FP32,
 * row-major, on the device of the network, read or written on its stream.
 * Every call returns a QUAPI_* code of quapi.h.
 */
#ifndef QUAPI_MLP_H
#define QUAPI_MLP_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct quapi_mlp quapi_mlp;

/* Create a network with parameters uniform in +-1/sqrt(fan_in), drawn from the
 * SplitMix64 sequence of seed, and buffers for batches up to max_batch.
 * stream: hipStream_t to run on, or NULL for a library stream.
 * Errors: EINVAL (a size < 1, n_in, width or n_out > 4096, depth > 64,
 * max_batch > 2^22), ENOMEM, EDEVICE. */
int quapi_mlp_create(int n_in, int width, int depth, int n_out, int max_batch, unsigned long long seed,
                     void* stream, quapi_mlp** out);

/* Number of parameters. */
int quapi_mlp_n_params(quapi_mlp* m, long long* n);

/* Copy the FP32 parameters in (host, n = n_params; the Adam state is reset) or
 * out; copy out the gradients of the last quapi_mlp_backward.  Synchronise. */
int quapi_mlp_set_params(quapi_mlp* m, const float* host, long long n);
int quapi_mlp_get_params(quapi_mlp* m, float* host, long long n);
int quapi_mlp_get_grads(quapi_mlp* m, float* host, long long n);

/* y = network(x) for 1 <= batch <= max_batch; enqueued on the stream. */
int quapi_mlp_forward(quapi_mlp* m, const float* x, int batch, float* y);

/* Forward and backward pass of the loss on (x, target): the gradients of the
 * loss with respect to every parameter into the network's gradient buffer, and
 * the loss into *loss (a device float; may be NULL).  Enqueued. */
int quapi_mlp_backward(quapi_mlp* m, const float* x, const float* target, int batch, float* loss);

/* One Adam step from the gradient buffer (bias-corrected, step count kept by
 * the network).  Errors: EINVAL (lr <= 0, beta outside [0, 1), eps <= 0). */
int quapi_mlp_adam(quapi_mlp* m, float lr, float beta1, float beta2, float eps);

/* Wait for the network's enqueued work. */
int quapi_mlp_sync(quapi_mlp* m);

/* Free the network (synchronises).  NULL is a no-op. */
void quapi_mlp_destroy(quapi_mlp* m);

#ifdef __cplusplus
}
#endif

#endif

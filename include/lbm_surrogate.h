/* Learned surrogate of the coupled 0D-3D solver: a multilayer perceptron
 * that maps the 7 parameters of the LV-elastance inlet, the Windkessel
 * outlet and the wall (Emax, Emin, HR, Z, C, R, k) to one beat of inlet
 * pressure and inlet flow, sampled at n_out / 2 phases each.
 *
 * The paper's coupled solver (the 0D fluid boundary equations, the direct
 * 0D-3D coupling and the fluid-structure algorithm of its Materials and
 * Methods) is what the network is trained to reproduce; the network itself
 * is this library's extension, not part of the paper.
 *
 * Network: h_0 = x_n (inputs mapped from the training box [lo, hi] onto
 * [-1, 1]); z_l = h_{l-1} W_l^T + b_l, h_l = GELU(z_l) (exact erf form) for
 * l = 1..n_hidden; y_n = h_L W^T + b; outputs y = mu + sigma * y_n.
 * Matrix products run on the gfx950 matrix cores with BF16 operands and FP32
 * accumulation; master weights, Adam moments and gradients are FP32.
 * Loss: mean over batch and outputs of (y_n - (t - mu) / sigma)^2.
 * Update: Adam with bias correction.
 *
 * Parameter vector layout (host and device): for each layer, W (out x in,
 * row-major) then b (out); layers 1..n_hidden+1.
 *
 * Memory: all device memory lives in one caller-owned buffer (size from
 * lbm_sur_query_sizes, 256-byte aligned) that must outlive the context.
 * Every call is enqueued on the stream given at init; calls that return
 * host data synchronise that stream.  Batch arrays are device pointers,
 * row-major FP32: x (m x n_in) physical parameters, t and y (m x n_out)
 * physical outputs.  An optional device index array idx (m int32, may be
 * NULL) selects the rows x[idx[r]], t[idx[r]] (a shuffled mini-batch
 * without a copy) out of the n_rows rows of x and t; an index outside
 * [0, n_rows) reads zeros and raises a device error flag that the next
 * synchronising call (lbm_sur_sync, or a loss read-back) reports as
 * LBM_E_INVAL.
 *
 * Errors: LBM_E_INVAL for a NULL or misaligned pointer, a size outside the
 * configured limits or a config that the kernels do not support (n_in > 32,
 * width and n_out multiples of 32); LBM_E_DEVICE for a HIP failure.
 * lbm_sur_last_error gives the message.
 */
#ifndef LBM_SURROGATE_H
#define LBM_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "lbm0d3d.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_sur_ctx lbm_sur_ctx;

typedef struct {
  int32_t n_in;        /* inputs (7) */
  int32_t width;       /* hidden width (512) */
  int32_t n_hidden;    /* hidden layers (4) */
  int32_t n_out;       /* outputs (512: 256 pressure then 256 flow phases) */
  int32_t max_batch;   /* rows per inference call */
  int32_t train_batch; /* rows per training or gradient call */
} lbm_sur_config;

/* Number of parameters (weights and biases) of the configured network. */
int64_t lbm_sur_num_params(const lbm_sur_config* cfg);

/* Bytes of device memory the context needs. */
lbm_status lbm_sur_query_sizes(const lbm_sur_config* cfg, size_t* bytes);

/* Create a context on the current device; mem is the device buffer. */
lbm_status lbm_sur_init(const lbm_sur_config* cfg, void* mem, size_t bytes, void* stream,
                        lbm_sur_ctx** out);

/* Load n = lbm_sur_num_params FP64 host values into the FP32 master weights
 * (rounded to nearest) and their BF16 copy; resets the Adam state. */
lbm_status lbm_sur_set_params(lbm_sur_ctx* c, const double* theta, int64_t n);
lbm_status lbm_sur_get_params(lbm_sur_ctx* c, double* theta, int64_t n);

/* Input box (n_in values each, lo < hi) and output standardisation (n_out
 * values each, sigma > 0), host arrays. */
lbm_status lbm_sur_set_scaling(lbm_sur_ctx* c, const double* lo, const double* hi, const double* mu,
                               const double* sigma);

/* Forward and backward pass on m <= train_batch rows without an update:
 * grad (device, num_params FP32) receives dLoss/dtheta; *loss (host, may
 * be NULL) the loss. */
lbm_status lbm_sur_grad(lbm_sur_ctx* c, const float* x, const float* t, int32_t n_rows, const int32_t* idx,
                        int32_t m, float* grad, double* loss);

/* One Adam step on m <= train_batch rows with learning rate lr and moments
 * (b1, b2, eps).  *loss (host, may be NULL: no synchronisation) receives
 * the loss before the step. */
lbm_status lbm_sur_train_step(lbm_sur_ctx* c, const float* x, const float* t, int32_t n_rows,
                              const int32_t* idx, int32_t m, double lr, double b1, double b2, double eps,
                              double* loss);

/* Inference: y (device, m x n_out FP32, physical units) for m <= max_batch
 * rows of x (physical parameters; no check of the box here: callers route
 * points outside it to the solver).  With width 512 and 512 outputs the
 * whole network runs as one kernel (activations stay on chip; the first
 * call after a weight change also rebuilds a fragment-ordered weight copy
 * in the context's memory); other shapes run one product per layer. */
lbm_status lbm_sur_predict(lbm_sur_ctx* c, const float* x, int32_t m, float* y);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * fused inference as lbm_sur_predict, with no context.  The network
 * (cfg->n_in <= 32, width 512, 1..7 hidden layers, 512 outputs;
 * max_batch and train_batch are not used) is read from the caller's device
 * arrays: theta (lbm_sur_num_params FP32 values in the parameter layout
 * above), the input box lo, hi (n_in FP32 each) and the output scaling mu,
 * sigma (n_out FP32 each); x (m x n_in) and y (m x 512) as for
 * lbm_sur_predict, 0 <= m <= 2^22.  All pointers device, 4-byte aligned,
 * owned by the caller; the work is enqueued on stream (NULL = default) and
 * nothing is synchronised.  With the same FP32 values (parameters and
 * scaling rounded to nearest from FP64, as lbm_sur_set_params and
 * lbm_sur_set_scaling do) the output equals lbm_sur_predict's bit for bit.
 * Scratch: the BF16 weights in fragment order go to a static device array
 * of 2^21 values (4 MiB) that each GPU holds for the life of the process;
 * every call rebuilds them from theta.  Calls on one GPU share that array,
 * so calls that overlap on one GPU (different streams, or host threads)
 * race.  Allocates nothing; its first call on a device looks up the array's
 * address there.  Errors: LBM_E_INVAL (NULL or misaligned pointer, a shape
 * the fused kernel does not take, m out of range), LBM_E_DEVICE (no
 * device, a failed launch); lbm_sur_last_error(NULL) gives the message of
 * this thread's last failed call. */
lbm_status lbm_sur_predict_static(const lbm_sur_config* cfg, const float* theta, const float* lo, const float* hi,
                                  const float* mu, const float* sigma, const float* x, int32_t m, float* y,
                                  void* stream);

/* Per-kernel time accumulation with HIP events on the context's stream
 * (matrix products and the fused inference kernel only): on/off, then
 * (launches, total ms, their FLOP count). */
lbm_status lbm_sur_set_timing(lbm_sur_ctx* c, int32_t on);
lbm_status lbm_sur_gemm_time(lbm_sur_ctx* c, int64_t* launches, double* ms, double* flops);

/* Wait for the context's stream and report (then clear) the device error
 * flag of an out-of-range index. */
lbm_status lbm_sur_sync(lbm_sur_ctx* c);

const char* lbm_sur_last_error(const lbm_sur_ctx* c);
lbm_status lbm_sur_destroy(lbm_sur_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* LBM_SURROGATE_H */

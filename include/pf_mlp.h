/*
 * pf_mlp.h -- C ABI of the learned pairwise capillary-bridge force surrogate on MI355X.
 *
 * A multilayer perceptron n_in -> hidden x layers -> 1 (SiLU activations) that maps the
 * parameters of a two-sphere bridge (surface gap, radius ratio, liquid volume, contact angle; the
 * quantities that fix the bridge of Sec. 2.2) to the capillary force along the line of centres.
 * Every matrix product of the forward and backward passes runs as a hand-written BF16 MFMA kernel
 * with FP32 accumulation; biases, activations, the loss and Adam run in FP32 on FP32 master
 * weights.  Inputs and targets are given already normalised by the caller.
 *
 * Conventions as in pf_lbm.h: the caller owns the device workspace, every call returns a status,
 * a handle binds to one stream, and a handle is not thread-safe.
 *
 * Parameter vector layout (FP32): for each layer l = 0 .. layers (the last maps to the output),
 * W_l [out][in] row-major then b_l [out].
 */
#ifndef PF_MLP_H
#define PF_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "pf_lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_mlp pf_mlp;

typedef struct {
    uint32_t struct_size; /* sizeof(pf_mlp_config)                                  */
    int32_t n_in;         /* inputs per sample, 1..16                                */
    int32_t hidden;       /* width of the hidden layers, 16..512, multiple of 16     */
    int32_t layers;       /* hidden layers, 1..8                                     */
    int32_t max_batch;    /* largest batch of any call, 1..65536                     */
} pf_mlp_config;

/* Create a network with parameters drawn from a seeded He-style uniform initialisation (biases
 * zero).  workspace == NULL: query mode (writes *ws_bytes_needed).  Errors as pf_lbm_init. */
int pf_mlp_init(const pf_mlp_config *cfg, uint64_t seed, void *workspace, size_t ws_bytes, void *hip_stream,
                pf_mlp **out, size_t *ws_bytes_needed);

/* Number of FP32 parameters. */
int32_t pf_mlp_num_params(const pf_mlp *h);

/* Replace / read the FP32 parameters (HOST arrays of pf_mlp_num_params floats).  Setting resets
 * the optimiser state.  Both synchronise the stream. */
int pf_mlp_set_params(pf_mlp *h, const float *params);
int pf_mlp_get_params(pf_mlp *h, float *params);

/* Forward pass: x DEVICE [n][n_in] FP32 -> y DEVICE [n] FP32, 1 <= n <= max_batch.  Async. */
int pf_mlp_forward(pf_mlp *h, const float *x, int32_t n, float *y);

/* Mean-squared-error loss over the batch and its gradient with respect to every parameter:
 * x DEVICE [n][n_in], t DEVICE [n] targets; grad HOST [num_params] FP32, loss HOST (may be
 * NULL).  Synchronises. */
int pf_mlp_gradients(pf_mlp *h, const float *x, const float *t, int32_t n, float *grad, double *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the mean-squared-error loss of the batch
 * with learning rate lr.  loss HOST may be NULL (then the call does not synchronise). */
int pf_mlp_train_step(pf_mlp *h, const float *x, const float *t, int32_t n, float lr, double *loss);

void pf_mlp_destroy(pf_mlp *h);
const char *pf_mlp_last_error(const pf_mlp *h);

#ifdef __cplusplus
}
#endif

#endif /* PF_MLP_H */

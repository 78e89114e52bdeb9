/*
 * Learned warm start for the dual potential (not in the paper): a small
 * network maps per-target features (y_j, source-blob centre c, width s,
 * log eps) to psi_j, so that Alg. 1 starts near the solution instead of at
 * zero. The paper's own starts (zero, eps schedule of Sec. 4.2, multilevel of
 * Sec. 5.3) stay as fallback and as the yardstick.
 *
 * Network: 6 inputs, 4 hidden layers of width 256 with the erf GELU, one
 * linear output; inputs are standardised per feature and the output is
 * de-standardised (mean/std held by the model). 199,425 parameters.
 *
 * Precision: FP32 master parameters and Adam moments; bfloat16 copies of the
 * weight matrices (round to nearest even, remade after every update); the
 * three 256x256 layers run on MFMA with bfloat16 operands and FP32
 * accumulation; hidden activations and the pre-activation gradients that feed
 * the matrix products are stored as bfloat16, everything else in FP32.
 * Training gradients are reduced in a fixed order: repeated calls give the
 * same bits.
 *
 * Flat parameter order (weight matrices [fan_in][fan_out], row-major):
 *   W0[6][256] b0[256] W1[256][256] b1[256] W2[256][256] b2[256]
 *   W3[256][256] b3[256] W4[256] b4[1]
 *
 * Memory: every pointer marked DEVICE is a device address on the model's
 * stream; HOST pointers are read or written before the call returns. The
 * model owns its parameters and a workspace that grows to the largest row
 * count seen (about 7.5 KB per row for training, 1 KB per row for inference).
 * Calls on one model must not overlap.
 */
#ifndef RSOT_MLP_H
#define RSOT_MLP_H

#include <stdint.h>

#include "rsot.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RSOT_MLP_IN 6
#define RSOT_MLP_WIDTH 256
#define RSOT_MLP_HIDDEN 4
#define RSOT_MLP_NPARAMS 199425

typedef struct rsot_mlp rsot_mlp;

/* Creates a model from FP32 parameters (HOST, RSOT_MLP_NPARAMS floats, flat
 * order above); normalisation starts as mean 0 / std 1. */
rsot_status rsot_mlp_create(const float *params, void *hip_stream, rsot_mlp **out);
void rsot_mlp_destroy(rsot_mlp *m);

/* Copies the parameters to HOST: which = 0 the FP32 masters, which = 1 the
 * values the kernels use (weight matrices rounded to bfloat16, biases FP32). */
rsot_status rsot_mlp_get_params(rsot_mlp *m, int which, float *params_out);

/* Replaces the masters (HOST) and resets the Adam moments and step count. */
rsot_status rsot_mlp_set_params(rsot_mlp *m, const float *params);

/* Input standardisation (feature - mean) / std and output de-standardisation
 * o * std + mean. HOST arrays of 6; every std must be > 0. */
rsot_status rsot_mlp_set_normalization(rsot_mlp *m, const float *feat_mean,
                                       const float *feat_std, float out_mean, float out_std);
rsot_status rsot_mlp_get_normalization(rsot_mlp *m, float *feat_mean, float *feat_std,
                                       float *out_mean, float *out_std);

/* Sets the normalisation to the mean and standard deviation (FP64 sums on
 * the device) of `rows` feature rows and targets (DEVICE). A feature of zero
 * spread gets std 1. */
rsot_status rsot_mlp_fit_normalization(rsot_mlp *m, const float *feats, const float *target,
                                       int64_t rows);

/* Feature rows (y0, y1, c0, c1, s, log eps) of n targets.
 *   y      DEVICE n x 2 doubles (row-major)
 *   cond   HOST 4 doubles: c0, c1, s, eps (eps > 0)
 *   feats  DEVICE n x 6 floats (out) */
rsot_status rsot_mlp_features(int64_t n, const double *y, const double *cond, float *feats,
                              void *hip_stream);

/* Prediction for `rows` feature rows (DEVICE rows x 6) into out (DEVICE
 * rows floats, de-standardised). rows = 0 is a no-op. */
rsot_status rsot_mlp_forward(rsot_mlp *m, const float *feats, int64_t rows, float *out);

/* Gradient of sum_r dout[r] * out[r] (out the de-standardised prediction)
 * with respect to every parameter, FP32 in flat order (DEVICE,
 * RSOT_MLP_NPARAMS floats). feats DEVICE rows x 6, dout DEVICE rows. */
rsot_status rsot_mlp_backward(rsot_mlp *m, const float *feats, int64_t rows, const float *dout,
                              float *grad);

/* One Adam step (Kingma & Ba) on the masters with gradient `grad` (DEVICE,
 * flat order); the step count is kept by the model. lr > 0, 0 <= b1, b2 < 1,
 * eps >= 0. The bfloat16 copies are remade. */
rsot_status rsot_mlp_adam_step(rsot_mlp *m, const float *grad, float lr, float b1, float b2,
                               float eps);

/* Forward, mean-squared-error loss in standardised output units
 * mean_r ((out_r - t_r) / out_std)^2, backward and one Adam step.
 *   feats   DEVICE table of feature rows (6 floats each)
 *   target  DEVICE table of targets (same row numbering)
 *   idx     DEVICE rows int64 row numbers into the tables, or NULL for 0..rows-1
 *   loss    HOST, the batch loss before the step; may be NULL (then no sync) */
rsot_status rsot_mlp_train_step(rsot_mlp *m, const float *feats, const float *target,
                                const int64_t *idx, int64_t rows, float lr, float b1, float b2,
                                float eps, double *loss);

/* Learned potential of n targets: features from y (DEVICE n x 2) and cond
 * (HOST c0, c1, s, eps), forward, then shifted in FP64 so that
 * sum_j nu_j psi_j = 0 (nu DEVICE). psi DEVICE n doubles (out). */
rsot_status rsot_mlp_predict_psi(rsot_mlp *m, int64_t n, const double *y, const double *nu,
                                 const double *cond, double *psi);

typedef struct {
    int used_learned;   /* 1: solved from the prediction; 0: fell back        */
    double predict_ms;  /* device time of the prediction                        */
    double J_pred;      /* J at the prediction (final eps); NaN if not finite   */
    double J_zero;      /* J at psi = 0 (final eps)                              */
} rsot_learned_info;

/*
 * Alg. 1 from the learned start: the prediction for the problem's targets
 * (2D problems only) is evaluated at the last eps of sp's schedule next to
 * psi = 0. If it is finite and gives the lower J, the solve runs at that eps
 * alone from the prediction; otherwise it runs sp's whole schedule from
 * zero. psi_out HOST n doubles (centred on success); info and linfo may be
 * NULL. sp->checkpoint is written as in rsot_solve; sp->resume is rejected
 * (INVALID_ARG): the start is the prediction. Errors as rsot_solve.
 */
rsot_status rsot_solve_learned(rsot_problem *p, rsot_mlp *m, const double *cond,
                               const rsot_solve_params *sp, double *psi_out, rsot_solve_info *info,
                               rsot_learned_info *linfo);

#ifdef __cplusplus
}
#endif

#endif /* RSOT_MLP_H */

/* Learned Newton initial guess for the FSI time step: C ABI.
 *
 * The Newton iteration of §3 (eq. (11)) starts each implicit step from a guess and judges
 * it by the nonlinear residual; the paper starts from the previous step's solution.  This
 * interface provides a better start without touching that test: a node-wise multilayer
 * perceptron, trained on the solver's own time steps, corrects the linear extrapolation
 *     g = 2 y_{n-1} - y_{n-2} + gain (*) sigma (*) MLP(x),
 * where x are per-vertex features of y_{n-1}, y_{n-2} and the inflow phase, (*) is the
 * componentwise product over the 7 components of a vertex, gain a per-component switch
 * (or weight) of the correction, and sigma the size of the last step's change:
 *     sigma[c] = max(sqrt((1/V) sum_i (y_{n-1} - y_{n-2})[i][c]^2), floor[c]).
 * Without a trained network the extrapolation alone is the guess.  A Newton solve reaches
 * the same residual tolerance from any guess, so the guess affects only the cost of the
 * step.
 *
 * Conventions: FP32 network, FP64 state vectors [V][7] as in fsi.h; device pointers are
 * the caller's and stay valid until the call returns; work runs on the stream given at
 * create time and calls return after it finished.  A call on zero rows (n = 0 or V = 0)
 * does nothing and accepts NULL arrays.  Errors are status codes (FSI_ERR_ARG for bad
 * arguments, FSI_ERR_HIP for a failed launch or copy), with a message from
 * fsi_mlp_last_error. */
#ifndef FSI_GUESS_H
#define FSI_GUESS_H

#include <stdint.h>

#include "fsi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsi_mlp fsi_mlp;

/* features per vertex: y1 / s (7), (y1 - y2) / sigma (7), 4 inflow-phase features */
#define FSI_GUESS_NIN 18

/* A perceptron with nlayers dense layers: nin -> hidden -> ... -> hidden -> nout, tanh
 * after every layer but the last.  Layer l has weights W_l [d_in][d_out] (row-major) and
 * bias b_l [d_out]; the parameter vector stores W_0, b_0, W_1, b_1, ... in order.  nmax is
 * the largest number of rows (vertices) one call may process; activations for nmax rows
 * are allocated here.  The parameters start undefined: set them with fsi_mlp_set_params. */
fsi_status fsi_mlp_create(int32_t nin, int32_t hidden, int32_t nlayers, int32_t nout, int64_t nmax,
                          void *hip_stream, fsi_mlp **out);
fsi_status fsi_mlp_destroy(fsi_mlp *m);
const char *fsi_mlp_last_error(const fsi_mlp *m);
int64_t fsi_mlp_nparams(const fsi_mlp *m);
/* (host) parameters in; resets the optimizer state (Adam moments and step count) */
fsi_status fsi_mlp_set_params(fsi_mlp *m, const float *params);
/* (host) parameters and/or the last computed gradient out (either pointer may be NULL) */
fsi_status fsi_mlp_get_params(fsi_mlp *m, float *params, float *grad);

/* Y [n][nout] = MLP(X [n][nin]), device, FP32 */
fsi_status fsi_mlp_forward(fsi_mlp *m, const float *X, int64_t n, float *Y);
/* mean squared error over the n * nout outputs against T [n][nout] (device), written to
 * *loss (host, may be NULL), and its gradient with respect to the parameters (kept for
 * fsi_mlp_get_params) */
fsi_status fsi_mlp_loss_grad(fsi_mlp *m, const float *X, const float *T, int64_t n, double *loss);
/* one Adam step (Kingma and Ba 2015, bias-corrected; lr > 0, 0 <= b1, b2 < 1) on the loss
 * of fsi_mlp_loss_grad; *loss is the loss before the step */
fsi_status fsi_mlp_train_step(fsi_mlp *m, const float *X, const float *T, int64_t n, float lr, float b1,
                              float b2, float eps, double *loss);

/* (host) the 21 scales: s [7] of y1, floor [7] of sigma, gain [7] of the output correction
 * (defaults 1, 0, 1) */
fsi_status fsi_mlp_set_scales(fsi_mlp *m, const float *scales);
/* X [V][FSI_GUESS_NIN] (device) from y1 = y_{n-1}, y2 = y_{n-2} (device [V][7]) and the
 * four inflow-phase features tfeat (host) */
fsi_status fsi_guess_features(fsi_mlp *m, const double *y1, const double *y2, int64_t V, const float *tfeat,
                              float *X);
/* training target T [V][7] = (y - (2 y1 - y2)) / sigma (device), sigma from (y1, y2) */
fsi_status fsi_guess_target(fsi_mlp *m, const double *y, const double *y1, const double *y2, int64_t V,
                            float *T);
/* guess [V][7] (device): the extrapolation corrected by the network (tfeat and the work
 * array Xwork [V][FSI_GUESS_NIN] given, V <= nmax), or the extrapolation alone (tfeat or
 * Xwork NULL) */
fsi_status fsi_guess_predict(fsi_mlp *m, const double *y1, const double *y2, int64_t V, const float *tfeat,
                             float *Xwork, double *guess);

/* C [M][ldc] = alpha A B + beta C on the matrix cores (FP32); A(m,k) = A[m*sam + k*sak],
 * B(k,n) = B[k*sbk + n*sbn] (device) -- the dense layers' GEMM, exposed for testing.
 * nsplit > 1 splits K over up to nsplit workgroups per 64x64 tile, with partial sums in
 * work (device, nsplit * M * N floats, caller-owned), added in a fixed order.  K = 0 gives
 * C = beta C, with A and B unused (may be NULL). */
fsi_status fsi_gemm_f32(int32_t M, int32_t N, int32_t K, float alpha, const float *A, int64_t sam, int64_t sak,
                        const float *B, int64_t sbk, int64_t sbn, float beta, float *C, int64_t ldc, int32_t nsplit,
                        float *work, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif

/*
 * rf_guess.h -- C ABI of the learned Picard initial guess on MI355X (gfx950).
 *
 * Not part of the paper's method: an extension of its Picard loop (Sec. 2.2,
 * 2.3), whose first iterate h^{n+1,0} is free (rf_step takes it as
 * h_guess_dev).  A small 3-D convolutional network predicts that iterate
 * from the state; plain Picard still runs to the same tolerance from it, so
 * the network changes how many iterations a step needs, never the answer's
 * tolerance.
 *
 * Network (all convolutions 3x3x3, zero padding outside the grid):
 *   features f (4 per cell): h^n / 10 m, (h^n - h^{n-1}) * 100 / m,
 *                            ln(Ks / Ks_layer), rain * 1e7 s/m
 *   z1 = conv(f; 4 -> 32) + b1, a1 = relu(z1)
 *   z2 = conv(a1; 32 -> 32) + b2, a2 = relu(z2)
 *   z3 = conv(a2; 32 -> 32) + b3, a3 = relu(z3)
 *   y  = conv(a3; 32 -> 1) + b4
 *   h^{n+1,0} = h^n + (h^n - h^{n-1}) + 0.01 m * y
 * i.e. the network corrects the linear extrapolation in time of the last
 * accepted increment (an untrained network, y = 0, returns that
 * extrapolation; h^{n-1} = h^n gives h^n plus the correction).
 * Weights are held in FP32 (the trained copy) and used as BF16; activations
 * are BF16, every product accumulates in FP32 (v_mfma_f32_16x16x32_bf16 on
 * the matrix cores; the 32 -> 1 layer with v_dot2_f32_bf16).  Training minimises the mean square of
 * (h^{n+1,0} - h^{n+1}) / 0.01 m over the grid against solver-converged
 * states, with hand-written backward kernels and Adam.
 *
 * Parameter vector (FP32, rf_guess_param_count values), layer by layer:
 * W_l[co][tap][ci] then b_l[co], tap = 9 (di+1) + 3 (dj+1) + (dk+1) for the
 * neighbour at (i+di, j+dj, k+dk); (Cin, Cout) = (4, 32), (32, 32),
 * (32, 32), (32, 1).
 *
 * Conventions as in rf.h: cell (i, j, k) of an nx*ny*nz grid is element
 * k + nz*(i + nx*j); device pointers belong to the caller; the library
 * allocates no device memory (the caller binds a workspace); work runs on
 * the stream given at creation; every call returns an rf_status.
 */
#ifndef RF_GUESS_H
#define RF_GUESS_H

#include "rf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rf_guess rf_guess;

rf_status rf_guess_create(rf_guess **out, int hip_device, void *hip_stream);
rf_status rf_guess_destroy(rf_guess *g);
const char *rf_guess_last_error(const rf_guess *g);

/* Grid the network runs on (any size; nz >= 1).  Resets the parameters to a
 * seeded initialisation (He-normal weights scaled per layer, zero biases;
 * the output layer starts at zero so that the untrained guess is h^n). */
rf_status rf_guess_setup(rf_guess *g, int nx, int ny, int nz, unsigned seed);
rf_status rf_guess_workspace_bytes(const rf_guess *g, size_t *bytes);
rf_status rf_guess_bind_workspace(rf_guess *g, void *dev, size_t bytes);

size_t rf_guess_param_count(void);
/* Copies the FP32 parameters in or out (host arrays of rf_guess_param_count
 * values); set also clears the Adam moments. */
rf_status rf_guess_set_params(rf_guess *g, const float *host);
rf_status rf_guess_get_params(const rf_guess *g, float *host);

/* h^{n+1,0} into guess_dev (device, N doubles) from h^n, h^{n-1} and the
 * ln Ks offsets (device, N doubles each; lnks may be NULL = zeros) and the
 * rain rate [m/s]. */
rf_status rf_guess_predict(rf_guess *g, const double *hn, const double *hprev, const double *lnks,
                           double rain, double *guess_dev);

/* Loss 0.5/N sum ((h^{n+1,0} - target) / 0.01 m)^2 and its gradient with respect
 * to the parameters (host array of rf_guess_param_count floats, may be NULL),
 * at the current parameters; no update. */
rf_status rf_guess_gradient(rf_guess *g, const double *hn, const double *hprev, const double *lnks,
                            double rain, const double *target, double *loss, float *grad_host);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * loss of one sample; *loss (may be NULL) receives the loss before the step. */
rf_status rf_guess_train_step(rf_guess *g, const double *hn, const double *hprev,
                              const double *lnks, double rain, const double *target, double lr,
                              double *loss);

#ifdef __cplusplus
}
#endif

#endif /* RF_GUESS_H */

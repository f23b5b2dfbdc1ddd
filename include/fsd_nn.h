/* Learned warm start for the Crank-Nicolson solves (extension; not part of
 * arXiv 2511.21198).  A four-level 3D convolution network corrects the
 * linear extrapolation in time 2 u^{m-1} - u^{m-2} of the next iterate, so
 * that PCG / PGMRES (Section 3) start closer to the solution; the solver's
 * plain initial guess u^{m-1} remains the fallback (FSD_X0_GUARDED in
 * fsd.h).  The Crank-Nicolson matrices do not depend on m, so the
 * extrapolation error is a linear map of du = u^{m-1} - u^{m-2} and
 * dF = F^{m-1/2} - F^{m-3/2}; these are the network's inputs.
 *
 * Network (all convolutions 3x3x3, zero padding, stride 1, with bias):
 *   features x = [du/s, dt dF/s, log(eta_1)/4, log(eta_2)/4, log(eta_3)/4],
 *            s = rms(du) + rms(dt dF) + 1e-30 (no history: du = 0,
 *            dF = F^{m-1/2});
 *   e0 = relu(conv 5->16)  e1 = relu(conv(pool e0) 16->32)
 *   e2 = relu(conv(pool e1) 32->64)  e3 = relu(conv(pool e2) 64->64)
 *   d2 = relu(conv(up e3 + e2) 64->32)  d1 = relu(conv(up d2 + e1) 32->16)
 *   y  = conv(up d1 + e0) 16->1;  guess = u^{m-1} + du + s y.
 * pool: 2x2x2 average, stride 2, size ceil(n/2) (absent inputs count as
 * zero); up: nearest neighbour.  Activations are bfloat16, convolutions run
 * on bf16 MFMA with float32 accumulation; parameters, gradients and Adam
 * state are float32 (caller-owned device arrays).
 *
 * Parameter vector: for the layers e0 e1 e2 e3 d2 d1 d0 in this order,
 * W[out][in][3][3][3] (C order, taps z-major) then b[out];
 * fsd_nn_param_count() floats in total.
 *
 * Grids: float64 inputs and outputs use the dense layout of fsd.h (x
 * fastest, [n3][n2][n1]); network inputs for training are float32
 * [batch][5][nz][ny][nx], targets and outputs float32 [batch][nz][ny][nx].
 * All work is enqueued on the bound stream (a hipStream_t passed as void*,
 * as in fsd.h); no function allocates device memory.  Errors: FSD_EINVAL
 * (bad sizes or null pointers), FSD_ENOTBOUND, FSD_ESMALLWS, FSD_EHIP. */
#ifndef FSD_NN_H
#define FSD_NN_H

#include "fsd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsd_nn_s* fsd_nn;

/* Number of float32 parameters. */
long fsd_nn_param_count(void);

/* Layer k (0..6 = e0 e1 e2 e3 d2 d1 d0): input and output channels, level. */
fsd_status fsd_nn_layer(int k, int* c_in, int* c_out, int* level);

/* A network instance for grids of nx x ny x nz voxels (each >= 1) and
 * `batch` grids per call; `training` != 0 adds the buffers of the backward
 * pass.  Host-only. */
fsd_status fsd_nn_create(int nx, int ny, int nz, int batch, int training, fsd_nn* out);
void fsd_nn_destroy(fsd_nn nn);
size_t fsd_nn_workspace_bytes(fsd_nn nn);
/* Binds a caller-owned device workspace (>= fsd_nn_workspace_bytes,
 * 256-byte aligned) and a stream. */
fsd_status fsd_nn_bind(fsd_nn nn, void* d_ws, size_t bytes, void* stream);

/* Features of one grid at step m (batch index 0; nx, ny, nz of the
 * instance): d_u = u^{m-1}, d_uprev = u^{m-2}, d_F = F^{m-1/2},
 * d_Fprev = F^{m-3/2}; d_x receives float32 [5][nz][ny][nx]; optional
 * training target d_t = (d_unext - 2 d_u + d_uprev) / s (d_unext = u^m) and
 * d_s (device double).  d_uprev, d_F, d_Fprev and d_unext may be NULL
 * (no history: du = 0 and the target uses u_prev = u; zero sources). */
fsd_status fsd_nn_features(fsd_nn nn, const double* d_u, const double* d_uprev, const double* d_F,
                           const double* d_Fprev, const double* d_unext, double dt,
                           const double eta[3], float* d_x, float* d_t, double* d_s);

/* Copies the box [x0, x0+cx) x [y0, y0+cy) x [z0, z0+cz) of each of the
 * c channels of d_src (float32 [c][nz][ny][nx]) to d_dst ([c][cz][cy][cx]). */
fsd_status fsd_nn_crop(const float* d_src, int c, int nx, int ny, int nz, int x0, int y0, int z0,
                       int cx, int cy, int cz, float* d_dst, void* stream);

/* y = network(x) for the batch. */
fsd_status fsd_nn_forward(fsd_nn nn, const float* d_params, const float* d_x, float* d_y);

/* Mean squared error over the interior (`margin` voxels dropped on every
 * side of every grid) between network(x) and d_t, into *d_loss (device
 * double), and its gradient with respect to the parameters into d_grad.
 * Needs a training instance. */
fsd_status fsd_nn_loss_grad(fsd_nn nn, const float* d_params, const float* d_x, const float* d_t,
                            int margin, float* d_grad, double* d_loss);

/* One Adam step (Kingma and Ba 2015), step count t >= 1:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
fsd_status fsd_nn_adam(long count, float* d_p, const float* d_g, float* d_m, float* d_v, int t,
                       double lr, double b1, double b2, double eps, void* stream);

/* guess = u + (u - u_prev) + s * network(features) on one full grid
 * (batch index 0); the arguments as in fsd_nn_features. */
fsd_status fsd_nn_predict(fsd_nn nn, const float* d_params, const double* d_u,
                          const double* d_uprev, const double* d_F, const double* d_Fprev,
                          double dt, const double eta[3], double* d_guess);

#ifdef __cplusplus
}
#endif

#endif

/*
 * libsde denoiser: the learned part beside the jump-SDE transport, C ABI.
 *
 * A fully convolutional 3D encoder-decoder maps a low-history dose map and
 * the density map to an estimate of the high-history dose map.  The paper
 * has no network (it is the learned extension of the dose engine of
 * section 2); it is trained only on pairs that the transport of sde.h
 * computes, and its output is accepted only where the gamma judge of
 * section 2.2 (sde_gamma) passes against a high-history reference.
 *
 * Network (levels L, base channels c0; channels c_l = c0 * 2^l):
 *   encoder level l: [2x2x2 average pool if l > 0] -> conv3 -> LReLU -> conv3 -> LReLU
 *   decoder level l = L-2..0: concat[skip_l, nearest-up(lower)] -> conv3 -> LReLU
 *                             -> conv3 -> LReLU
 *   head: 1x1x1 conv to one channel, plus the input dose (residual)
 * conv3 = 3x3x3 cross-correlation, zero padding 1, weights [co][t][ci] with
 * tap t = 9(dz+1) + 3(dy+1) + (dx+1), plus bias.  Input channels: 0 the
 * normalised dose, 1 the density, 2..cin-1 zero.
 *
 * Arithmetic: activations and conv weights bf16 (round to nearest even),
 * products accumulated in FP32 on the matrix cores; loss, gradients of the
 * activations, master weights and Adam moments FP32.  All reductions run in
 * a fixed order: training is bit-reproducible.
 *
 * Parameters are one FP32 vector in this order: for l = 0..L-1 enc{l}a,
 * enc{l}b; for l = L-2..0 dec{l}a, dec{l}b; each conv as weight
 * [co][27][ci] then bias [co]; then head weight [c0] and head bias [1].
 *
 * Conventions as in sde.h: 0 or a negative sde_status; sde_last_error()
 * explains the last failure; work runs on the stream of sde_set_stream;
 * (device) arrays are the caller's, C-contiguous.  Volumes passed to the
 * network are [B][D][H][W] with D, H, W multiples of 2^(L-1).
 */
#ifndef SDE_NN_H
#define SDE_NN_H

#include <stddef.h>
#include <stdint.h>

#include "sde.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sde_nn sde_nn;

typedef struct {
    int levels;          /* L, 1..5 */
    int base_channels;   /* c0: 16 or 32 */
    int in_channels;     /* cin: multiple of 16 (2 used, the rest zero) */
    float leaky_alpha;   /* LeakyReLU slope below zero, > 0 */
    int max_batch;       /* buffer sizes: B, D, H, W of the largest call */
    int max_d, max_h, max_w;
    int train;           /* nonzero: allocate gradient, Adam and loss buffers */
    float adam_beta1, adam_beta2, adam_eps;
    int store_concat;    /* nonzero: each decoder level stores concat[skip, up(lower)]
                            before its conv; zero: the convs (and in training the
                            weight gradients) read it in place where they support
                            the shape (the same sums in the same order either way) */
} sde_nn_config;

/* Create a network; parameters start at zero (set them with
 * sde_nn_set_params).  Allocates all device buffers for the maximum sizes. */
int sde_nn_create(const sde_nn_config* cfg, sde_nn** out);
int sde_nn_destroy(sde_nn* net);
/* Number of FP32 parameters. */
int sde_nn_param_count(const sde_nn* net, int64_t* n_out);
/* Copy FP32 master parameters in/out (host arrays of param_count floats);
 * set also refreshes the bf16 copy the kernels read. */
int sde_nn_set_params(sde_nn* net, const float* params, int64_t n);
int sde_nn_get_params(sde_nn* net, float* params, int64_t n);
/* Adam state for checkpoint and resume (host arrays of param_count floats,
 * step = number of updates taken). */
int sde_nn_set_adam_state(sde_nn* net, const float* m, const float* v, int64_t n, int64_t step);
int sde_nn_get_adam_state(sde_nn* net, float* m, float* v, int64_t n, int64_t* step);
/* Gradient of the last sde_nn_loss_grad call (host array of param_count floats). */
int sde_nn_get_grads(sde_nn* net, float* grads, int64_t n);

/* Forward pass.  dose, rho (nullable), out: (device) FP32 [B][D][H][W]. */
int sde_nn_forward(sde_nn* net, const float* dose, const float* rho, int B, int D, int H, int W,
                   float* out);
/* Forward, loss = mean(m (out - target)^2) (m = weight, nullable = 1) and
 * the gradient of every parameter (kept on the device).  loss_out (host)
 * receives the loss; the call synchronises the stream.  Needs train. */
int sde_nn_loss_grad(sde_nn* net, const float* dose, const float* rho, const float* target,
                     const float* weight, int B, int D, int H, int W, float* loss_out);
/* One Adam update (Kingma and Ba) with the gradient of the last
 * sde_nn_loss_grad and learning rate lr; refreshes the bf16 weights. */
int sde_nn_adam_step(sde_nn* net, float lr);

/* Denoise one dose grid: dose (device, FP64 [nz][ny][nx], e.g. the output
 * of sde_transport) is divided by its maximum, zero padded to multiples of
 * 2^(L-1), passed with the density (device FP32 [nz][ny][nx], nullable)
 * through the network, clamped at zero, cropped and multiplied back into
 * out (device FP64 [nz][ny][nx]; may alias dose). */
int sde_nn_denoise(sde_nn* net, const double* dose, const float* rho, int nx, int ny, int nz,
                   double* out);

/* Training pair from two dose grids of the same beam (device FP64, n
 * voxels): m = max |low|; low_out = low / m, high_out = high / m (high
 * nullable) and the loss weight weight_out (nullable): with h =
 * max(high_out, 0), 1 / (h + eps)^2 where h >= thr (relative error with a
 * floor of eps) and (h / thr) / (thr + eps)^2 below thr (fading out where a
 * gamma test with threshold thr does not look).  Outputs are device FP32.
 * Uses the network's scratch for m. */
int sde_nn_prepare_pair(sde_nn* net, const double* low, const double* high, int64_t n, float eps,
                        float thr, float* low_out, float* high_out, float* weight_out);

/* Single layers, for tests of the kernels.  x, w, y16, dz: (device) bf16
 * bit patterns (uint16); bias, y32, dx, dw, db: (device) FP32.
 * Volumes [B][D][H][W][C]; weights [Co][27][Ci].  Ci % 16 == 0 and
 * Co / 16 in {1, 2, 3, 4, 6, 8, 12}.  bf16 arrays and workspaces must be
 * 16-byte aligned (SDE_E_INVALID otherwise). */
/* y = act(conv3(x, w) + bias) into y16 and/or y32 (either nullable); act 0/1. */
int sde_nn_conv3d_fwd(const uint16_t* x, const uint16_t* w, const float* bias, int B, int D,
                      int H, int W, int Ci, int Co, float alpha, int act, uint16_t* y16,
                      float* y32);
/* Workspace bytes that sde_nn_conv3d_dgrad / _wgrad need for these sizes. */
int sde_nn_conv3d_workspace(int B, int D, int H, int W, int Ci, int Co, size_t* bytes);
/* dx[v][ci] = sum_t sum_co dz[v - off(t)][co] w[co][t][ci] (FP32 out). */
int sde_nn_conv3d_dgrad(const uint16_t* dz, const uint16_t* w, int B, int D, int H, int W, int Ci,
                        int Co, float* dx, void* workspace, size_t workspace_bytes);
/* dw[co][t][ci] = sum_v dz[v][co] x[v + off(t)][ci]; db[co] = sum_v dz[v][co] (nullable).
 * Also needs (Co / 16) * (Ci / 16) <= 64. */
int sde_nn_conv3d_wgrad(const uint16_t* dz, const uint16_t* x, int B, int D, int H, int W, int Ci,
                        int Co, float* dw, float* db, void* workspace, size_t workspace_bytes);

#ifdef __cplusplus
}
#endif

#endif /* SDE_NN_H */

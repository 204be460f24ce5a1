// Launchers of the denoiser kernels (nn_kernels.hip), used by nn_api.cpp.
// Volumes are channels-last [B][D][H][W][C]; dims = {B, D, H, W}.  bf16
// values travel as uint16_t bit patterns.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sde {
namespace nn {

// 3x3x3 conv, zero padding 1; y = act(conv(x, w) + bias) to bf16 y16 and/or
// FP32 y32 (y32 += result when accumulate).  Ci % 16 == 0, Co % 16 == 0 and
// Co / 16 in {1, 2, 3, 4, 6, 8, 12}.  bias may be null; act = LeakyReLU(alpha).
// The kernel is chosen by the channel counts: registers-held weights for
// Ci <= 48 with 16 or 32 outputs, 32-channel passes for Ci >= 64 with 32 or
// 64, LDS weight slabs otherwise.
//
// With ym non-null (bias, act, accumulate and y32 zero) y16 gets instead the
// input gradient of a LeakyReLU layer whose output is ym (Co channels):
// bf16(ym > 0 ? r : alpha r), r the FP32 conv output, what lrelu_bwd turns
// it into; only where conv_dz_wide_supported(Ci, Co, dims) holds.
hipError_t conv_fwd(const uint16_t* x, const uint16_t* w, const float* bias, const int* dims,
                    int Ci, int Co, float alpha, int act, uint16_t* y16, float* y32,
                    int accumulate, hipStream_t s, const uint16_t* ym = nullptr);
bool conv_dz_wide_supported(int Ci, int Co, const int* dims);
// conv_fwd (bf16 output) of the decoder input concat[skip (Cs channels),
// nearest-up(low) (Cu channels, half size)] without storing the
// concatenation; only the shapes and sizes (nvox voxels at the skip level)
// conv_cat_fwd_supported accepts.
bool conv_cat_fwd_supported(int Cs, int Cu, int Co, long long nvox);
hipError_t conv_cat_fwd(const uint16_t* skip, const uint16_t* low, const uint16_t* w,
                        const float* bias, const int* dims, int Cs, int Cu, int Co, float alpha,
                        int act, uint16_t* y16, hipStream_t s);
// The last decoder conv (16 -> 16, LeakyReLU) with the head fused in: y16
// (nullable) as conv_fwd stores it, and out[v] = head_b + resid[v] +
// sum_c head_w[c] y16[v][c] summed per 4 channels, the four partial sums
// added pairwise.
hipError_t conv_head_fwd(const uint16_t* x, const uint16_t* w, const float* bias, const int* dims,
                         float alpha, uint16_t* y16, const float* head_w, const float* head_b,
                         const float* resid, float* out, hipStream_t s);
// The first layer's conv_fwd (16 outputs, LeakyReLU, bf16 output) from the
// input's two used channels as bf16 pairs x2 (weights [16][27][cin]).
hipError_t conv_in_fwd(const uint32_t* x2, const uint16_t* w, int cin, const float* bias,
                       const int* dims, float alpha, uint16_t* y16, hipStream_t s);
// The input gradient of the level-0 decoder conv (Ci = 16, Co = 48, cs = 16):
// conv_fwd without bias or activation, its output channels split.  [0, cs)
// go in FP32 into ya (cs per voxel) when ya is non-null (else the caller
// takes them later with conv_dz_fwd); [cs, Co), the upsampled half, go
// through the upsampling backward and the LeakyReLU of the level below:
// dzc (bf16, half size, Co - cs per voxel) gets what up_bwd with target
// activation ym (half size, Co - cs per voxel) and alpha gives.  D, H, W
// even; dzc must not be x.
hipError_t conv_fwd_split(const uint16_t* x, const uint16_t* w, const int* dims, int Ci, int Co,
                          int cs, float* ya, const uint16_t* ym, float alpha, uint16_t* dzc,
                          hipStream_t s);
// conv_fwd 16 -> 16 (LeakyReLU, bf16 y16) with pool_fwd of its output fused
// in: pool (bf16, half size; D, H, W even) gets the values pool_fwd gives.
hipError_t conv_pool_fwd(const uint16_t* x, const uint16_t* w, const float* bias, const int* dims,
                         float alpha, uint16_t* y16, uint16_t* pool, hipStream_t s);
// The input gradient of a LeakyReLU layer through the next conv (16 -> 16):
// dz = bf16(ym > 0 ? r : alpha r), r = conv(x, w) in FP32 (no bias); the same
// values as conv_fwd into FP32 followed by lrelu_bwd.  With par non-null (the
// gradient of the pooled layer, FP32, half size, 16 channels; D, H, W even)
// r = conv(x, w) + par[parent] / 8: conv_fwd into FP32 followed by pool_bwd
// with a LeakyReLU target.  dz must not be x.
hipError_t conv_dz_fwd(const uint16_t* x, const uint16_t* w, const int* dims, const uint16_t* ym,
                       float alpha, uint16_t* dz, hipStream_t s, const float* par = nullptr);
// flip_transpose of several layers in one launch
constexpr int kMaxFlipJobs = 32;
struct FlipJobs {
    int n = 0;
    const uint16_t* w[kMaxFlipJobs];
    uint16_t* wt[kMaxFlipJobs];
    int ci[kMaxFlipJobs], co[kMaxFlipJobs];
    long long start[kMaxFlipJobs + 1];
};
hipError_t flip_transpose_all(const FlipJobs& jobs, hipStream_t s);
// wt[ci][26 - t][co] = w[co][t][ci] (weights of the input-gradient conv)
hipError_t flip_transpose(const uint16_t* w, uint16_t* wt, int Ci, int Co, hipStream_t s);
// weight gradient: part needs wgrad_part_floats floats; dw [Co][27][Ci], db [Co]
// (nullable).  Ci % 16 == 0, Co % 16 == 0, (Co/16)(Ci/16) <= 64, chunk from
// wgrad_chunk_for (a multiple of 64).  16, 32, 64 or 128 outputs go by
// 4 x 4 x 16 bricks (at most as many split-K chunks as the chunk length
// gives; 64 and 128 as groups of 32), other widths by 64-voxel slices and
// tap groups.
long long wgrad_chunks(const int* dims, int chunk);
int wgrad_chunk_for(const int* dims, int Ci, int Co, long long max_part_floats);
long long wgrad_part_floats(const int* dims, int Ci, int Co, int chunk);
hipError_t wgrad(const uint16_t* dz, const uint16_t* x, const int* dims, int Ci, int Co, int chunk,
                 float* part, float* dw, float* db, hipStream_t s);
// wgrad of a conv whose input is the decoder's concatenation [skip (Cs
// channels), nearest-upsampled low (Cu channels, half-size level)], read in
// place.  Supported (by bricks) when wgrad_cat_supported says so; the part
// buffer is sized as for wgrad with Ci = Cs + Cu.
bool wgrad_cat_supported(int Cs, int Cu, int Co, const int* dims);
hipError_t wgrad_cat(const uint16_t* dz, const uint16_t* skip, const uint16_t* low,
                     const int* dims, int Cs, int Cu, int Co, int chunk, float* part, float* dw,
                     float* db, hipStream_t s);
hipError_t lrelu_bwd(const float* dy, const uint16_t* y, float alpha, long long n, uint16_t* dz,
                     hipStream_t s);
hipError_t pool_fwd(const uint16_t* x, const int* dims_out, int C, uint16_t* y, hipStream_t s);
// pool_bwd / up_bwd: with dz non-null the FP32 result is not stored; it goes
// through the LeakyReLU derivative of y (the activation it is the gradient
// of, same layout) into dz (bf16), as lrelu_bwd would turn it.  pool_bwd's
// dx holds cx channels per voxel (0: C), of which the first C are added to.
hipError_t pool_bwd(const float* dy, const int* dims_in, int C, float* dx, hipStream_t s,
                    const uint16_t* y = nullptr, float alpha = 0.0f, uint16_t* dz = nullptr,
                    int cx = 0);
hipError_t up_fwd(const uint16_t* x, const int* dims_fine, int C, int Cf, int c0, uint16_t* y,
                  hipStream_t s);
hipError_t up_bwd(const float* dy, const int* dims_coarse, int C, int Cf, int c0, float* dx,
                  hipStream_t s, const uint16_t* y = nullptr, float alpha = 0.0f,
                  uint16_t* dz = nullptr);
hipError_t copy_channels(const uint16_t* x, const int* dims, int C, int Cf, int c0, uint16_t* y,
                         hipStream_t s);
// network input from normalised FP32 maps (rho nullable): channel 0 dose,
// channel 1 density, the rest zero, as Cx-channel rows x (nullable) and as
// bf16 pairs x2[v] = dose | density << 16 (nullable); resid = dose
hipError_t assemble_f32(const float* dose, const float* rho, long long nv, int Cx, uint16_t* x,
                        uint32_t* x2, float* resid, hipStream_t s);
// network input from a dose grid [nz][ny][nx] (FP64) divided by *maxp, zero
// padded into [D][H][W]; rho (FP32, nullable) padded likewise
hipError_t assemble_grid(const double* dose, const float* rho, const int* src, const int* dst,
                         const double* maxp, int Cx, uint16_t* x, uint32_t* x2, float* resid,
                         hipStream_t s);
// out (FP64 [nz][ny][nx]) = max(0, net[D][H][W] cropped) * (*maxp)
hipError_t finish_grid(const float* net, const int* src, const int* dst, const double* maxp,
                       double* out, hipStream_t s);
// lo = low / *maxp, hi = high / *maxp (high nullable); wt = 1 / (h + eps)^2 for
// h = max(hi, 0) >= thr, else (h / thr) / (thr + eps)^2
hipError_t prepare_pair(const double* low, const double* high, long long n, const double* maxp,
                        float eps, float thr, float* lo, float* hi, float* wt, hipStream_t s);
hipError_t max_abs(const double* a, long long n, unsigned long long* out_bits, hipStream_t s);
hipError_t head_fwd(const uint16_t* x, const float* w, const float* b, const float* resid,
                    long long nv, int C, float* out, hipStream_t s);
int head_bwd_blocks(long long nv);
// head backward: dx = dout w (FP32), or with dz non-null the gradient through
// the LeakyReLU that produced x, dz = bf16(x > 0 ? dout w : alpha dout w)
// (lrelu_bwd's values) in place of dx; per-block partials of dw and db
hipError_t head_bwd(const float* dout, const uint16_t* x, const float* w, long long nv, int C,
                    float* dx, float* part, hipStream_t s, float alpha = 0.0f,
                    uint16_t* dz = nullptr);
int mse_blocks(long long n);
hipError_t mse(const float* out, const float* tgt, const float* wgt, long long n, float* dout,
               float* part, hipStream_t s);
// out[c] = sum_r part[r * ncol + c] for r < nrow (fixed order)
hipError_t sum_rows(const float* part, int nrow, int ncol, float* out, hipStream_t s);
hipError_t adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1,
                float b2, float eps, int step, uint16_t* p16, hipStream_t s);
hipError_t f32_to_bf16(const float* a, long long n, uint16_t* b, hipStream_t s);
hipError_t fill_u32(uint32_t* p, long long n, uint32_t v, hipStream_t s);

}  // namespace nn

// the library's current stream and error reporting (sde_api.cpp)
hipStream_t library_stream();
int report_error(int code, const char* msg);

}  // namespace sde

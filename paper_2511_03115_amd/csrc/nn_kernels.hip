// HIP kernels of the dose denoiser for gfx950: a 3D convolutional
// encoder-decoder trained and run entirely on these kernels.
//
// Tensors are channels-last volumes [B][D][H][W][C]; activations and conv
// weights are bf16, accumulation FP32 on the matrix cores
// (v_mfma_f32_16x16x32_bf16), gradients and master weights FP32.
//
// MFMA 16x16x32 bf16 operand layout (lane l of a wave64, i = 0..7 / 0..3):
//   A[m = l%16][k = (l/16)*8 + i],  B[k = (l/16)*8 + i][n = l%16],
//   D[m = (l/16)*4 + i][n = l%16].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "nn_internal.hpp"

namespace sde {
namespace nn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float -> bf16, round to nearest even (the hardware conversion)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
// two floats rounded to bf16 (as f2bf) in one conversion: a | b << 16
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

// LeakyReLU; for a slope in (0, 1] it is max(r, alpha r)
__device__ __forceinline__ float lrelu(float r, float alpha) {
    return alpha <= 1.0f ? fmaxf(r, alpha * r) : (r > 0.0f ? r : alpha * r);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// Raw buffer resource over n bf16 elements (gfx9 descriptor word 3: 32-bit
// data format; a zero format reads zeros).  n * 2 must stay below 2^31.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc16(const uint16_t* p, long long n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(p), 0, (int)(n * 2), 0x00020000);
}

// 16-byte buffer load at byte offset off, or zeros when !ok (then offset 0
// is read, which is always in range, and discarded).
__device__ __forceinline__ uint4 ld16(__amdgpu_buffer_rsrc_t r, int off, bool ok) {
    const uint4 v =
        __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, ok ? off : 0, 0, 0));
    return ok ? v : make_uint4(0, 0, 0, 0);
}

struct Geo {
    int B, D, H, W;
    __host__ __device__ __forceinline__ long long nvox() const { return (long long)B * D * H * W; }
};

// ---------------------------------------------------------------------------
// conv3d 3x3x3, zero padding 1, stride 1: y[v][co] = act(bias[co] +
//   sum_{t, ci} x[shift(v, t)][ci] w[co][t][ci]), as an implicit GEMM with
// M = voxels, N = Co, K = 27 Ci (k = t*Ci + ci), outputs bf16 (optional)
// and/or FP32 (optional, added to when accumulate).  The K dimension
// (k = t*Ci + ci) is walked in slabs of kSlab: the workgroup copies
// W[:, slab] into LDS ([co][kSlab + 8] bf16; the 16-byte row pad puts the 16
// rows a quarter-wave reads on distinct banks), then every wave multiplies
// MT 16-voxel row tiles by all NT 16-channel column tiles, so each weight
// fragment read from LDS feeds MT matrix-core ops and each gathered input
// fragment feeds NT.  Voxel coordinates are decoded once per kernel and
// the (tap, channel) position of each lane advances incrementally.
// blockIdx.y selects the group of NT column tiles (output channels from
// 16 NT blockIdx.y), so a small volume can spread its columns over several
// workgroups.
// ---------------------------------------------------------------------------
constexpr int kSlab = 128;
constexpr int kSlabRow = kSlab + 8;

template <int NT, int MT>
__global__ void __launch_bounds__(256) k_conv_fwd_lds(const uint16_t* __restrict__ x,
                                                      const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias, Geo g,
                                                      int Ci, int Co, float alpha, int act,
                                                      uint16_t* __restrict__ y16,
                                                      float* __restrict__ y32, int accumulate) {
    extern __shared__ __align__(16) uint16_t wl[];   // [NT*16][kSlabRow]
    const int lane = threadIdx.x & 63;
    const int cob = blockIdx.y * NT * 16;             // first output channel of this block
    const long long nv = g.nvox();
    const long long base = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * (16 * MT);
    const int K = 27 * Ci;
    // this lane's A rows: voxel coordinates, decoded once
    int vx[MT], vy[MT], vz[MT];
    bool ok[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const long long v = base + m * 16 + (lane & 15);
        ok[m] = v < nv;
        const long long vv = ok[m] ? v : 0;
        vx[m] = (int)(vv % g.W);
        vy[m] = (int)((vv / g.W) % g.H);
        vz[m] = (int)((vv / ((long long)g.W * g.H)) % g.D);
    }
    const long long plane = (long long)g.W * g.H;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // (tap, channel) of this lane's first k: k = (lane / 16) * 8
    int t = ((lane >> 4) * 8) / Ci;
    int ci = ((lane >> 4) * 8) - t * Ci;
    const int rows = NT * 16;
    for (int k0 = 0; k0 < K; k0 += kSlab) {
        __syncthreads();
        for (int i = threadIdx.x; i < rows * (kSlab / 8); i += blockDim.x) {
            const int r = i / (kSlab / 8), c = (i - r * (kSlab / 8)) * 8;
            uint4 val = make_uint4(0, 0, 0, 0);
            if (cob + r < Co && k0 + c < K)
                val = *reinterpret_cast<const uint4*>(w + (size_t)(cob + r) * K + k0 + c);
            *reinterpret_cast<uint4*>(wl + r * kSlabRow + c) = val;
        }
        __syncthreads();
        for (int kc = 0; kc < kSlab && k0 + kc < K; kc += 32) {
            const int kk = kc + (lane >> 4) * 8;
            const bool kin = k0 + kk < K;
            bf16x8 a[MT];
            const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                uint4 av = make_uint4(0, 0, 0, 0);
                const int xs = vx[m] + dx, ys = vy[m] + dy, zs = vz[m] + dz;
                if (kin && ok[m] && xs >= 0 && ys >= 0 && zs >= 0 && xs < g.W && ys < g.H &&
                    zs < g.D) {
                    const long long sv = base + m * 16 + (lane & 15) + dx + (long long)dy * g.W +
                                         dz * plane;
                    av = *reinterpret_cast<const uint4*>(x + sv * Ci + ci);
                }
                a[m] = as_bf16x8(av);
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const uint4 bv =
                    *reinterpret_cast<const uint4*>(wl + (j * 16 + (lane & 15)) * kSlabRow + kk);
                const bf16x8 b = as_bf16x8(bv);
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b, acc[m][j], 0, 0, 0);
            }
            ci += 32;
            while (ci >= Ci) {
                ci -= Ci;
                ++t;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = cob + j * 16 + (lane & 15);
        if (co >= Co) continue;
        const float b = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long v = base + m * 16 + (lane >> 4) * 4 + i;
                if (v >= nv) continue;
                float r = acc[m][j][i] + b;
                if (act) r = lrelu(r, alpha);
                if (y16) y16[v * Co + co] = f2bf(r);
                if (y32) y32[v * Co + co] = accumulate ? y32[v * Co + co] + r : r;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The same convolution for few input channels (Ci <= 48) and outputs (NT <=
// 2 column tiles), where the input gathers dominate: a workgroup computes a
// 4 x 8 x 8 brick of output voxels and first stages the 6 x 10 x 10 input
// brick with its one-voxel halo in LDS ([voxel][Ci + 8]; the 16-byte pad
// puts the 16 voxels a quarter-wave reads on distinct banks), so each input
// voxel is read from memory about 2.3 times instead of 27.  Wave w owns
// z-slice w of the brick as 4 row tiles of 16 voxels (two 8-voxel rows
// each).  Weights are staged in slabs as in k_conv_fwd_lds.  The register
// and channel-pass kernels below replace it where they apply; it remains
// for the other few-channel shapes (e.g. 48 inputs with 32 outputs) and for
// operands of 2 GiB or more, beyond their 32-bit buffer offsets.
// ---------------------------------------------------------------------------
constexpr int kHZ = 4, kHY = 8, kHX = 8;
constexpr int kHVox = (kHZ + 2) * (kHY + 2) * (kHX + 2);

// Brick of the register, row-reuse and channel-pass kernels below: 4 x 4 x
// 16 output voxels, so a 16-voxel matrix row is one run along x.
constexpr int kRZ = 4, kRY = 4, kRX = 16;
constexpr int kRVox = (kRZ + 2) * (kRY + 2) * (kRX + 2);

// Elements per voxel slot of the row-reuse kernel's brick in LDS.  Its
// matrix-core fragment reads are 16 voxels x 4 lane quarters x 16 bytes;
// gfx950 serves them at its full 256 bytes per clock when consecutive voxel
// slots are 32 or 96 bytes apart, and at half rate for 48, 64, 80 or 112
// (measured on the device for every K step's fragment pattern), so 32
// channels are padded to 48 and 16 or 48 channels are not padded.  (The
// register and channel-pass kernels keep a 16-byte pad per slot: in them the
// unpadded layout measured no faster.)
__host__ __device__ constexpr int brick_row(int ci) { return ci == 32 ? 48 : ci; }

template <int NT>
__global__ void __launch_bounds__(256) k_conv_fwd_halo(const uint16_t* __restrict__ x,
                                                       const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias, Geo g,
                                                       int Ci, int Co, float alpha, int act,
                                                       uint16_t* __restrict__ y16,
                                                       float* __restrict__ y32, int accumulate) {
    constexpr int MT = 4;
    extern __shared__ __align__(16) uint16_t sm[];
    const int row = Ci + 8;
    uint16_t* hx = sm;                           // [kHVox][row]
    uint16_t* wl = sm + kHVox * row;             // [NT*16][kSlabRow]
    const int K = 27 * Ci;
    const int nbx = (g.W + kHX - 1) / kHX, nby = (g.H + kHY - 1) / kHY, nbz = (g.D + kHZ - 1) / kHZ;
    int bid = blockIdx.x;
    const int bx = bid % nbx;
    bid /= nbx;
    const int by = bid % nby;
    bid /= nby;
    const int bz = bid % nbz;
    const int b = bid / nbz;
    const int x0 = bx * kHX, y0 = by * kHY, z0 = bz * kHZ;
    const int gv = Ci / 8;
    for (int i = threadIdx.x; i < kHVox * gv; i += blockDim.x) {
        const int hv = i / gv, c = (i - hv * gv) * 8;
        const int hxx = hv % (kHX + 2), hyy = (hv / (kHX + 2)) % (kHY + 2),
                  hzz = hv / ((kHX + 2) * (kHY + 2));
        const int xx = x0 - 1 + hxx, yy = y0 - 1 + hyy, zz = z0 - 1 + hzz;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (xx >= 0 && yy >= 0 && zz >= 0 && xx < g.W && yy < g.H && zz < g.D) {
            const long long v = (((long long)b * g.D + zz) * g.H + yy) * g.W + xx;
            val = *reinterpret_cast<const uint4*>(x + v * Ci + c);
        }
        *reinterpret_cast<uint4*>(hx + hv * row + c) = val;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int hb[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int ly = 2 * m + ((lane & 15) >> 3), lx = lane & 7;
        hb[m] = ((wave + 1) * (kHY + 2) + (ly + 1)) * (kHX + 2) + (lx + 1);
    }
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    int t = ((lane >> 4) * 8) / Ci;
    int ci = ((lane >> 4) * 8) - t * Ci;
    const int rows = NT * 16;
    for (int k0 = 0; k0 < K; k0 += kSlab) {
        __syncthreads();   // (first pass: also orders the halo stores)
        for (int i = threadIdx.x; i < rows * (kSlab / 8); i += blockDim.x) {
            const int r = i / (kSlab / 8), c = (i - r * (kSlab / 8)) * 8;
            uint4 val = make_uint4(0, 0, 0, 0);
            if (r < Co && k0 + c < K)
                val = *reinterpret_cast<const uint4*>(w + (size_t)r * K + k0 + c);
            *reinterpret_cast<uint4*>(wl + r * kSlabRow + c) = val;
        }
        __syncthreads();
        for (int kc = 0; kc < kSlab && k0 + kc < K; kc += 32) {
            const int kk = kc + (lane >> 4) * 8;
            const bool kin = k0 + kk < K;
            const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
            const int off = (dz * (kHY + 2) + dy) * (kHX + 2) + dx;
            bf16x8 a[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                uint4 av = make_uint4(0, 0, 0, 0);
                if (kin) av = *reinterpret_cast<const uint4*>(hx + (hb[m] + off) * row + ci);
                a[m] = as_bf16x8(av);
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const uint4 bv =
                    *reinterpret_cast<const uint4*>(wl + (j * 16 + (lane & 15)) * kSlabRow + kk);
                const bf16x8 bb = as_bf16x8(bv);
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bb, acc[m][j], 0, 0, 0);
            }
            ci += 32;
            while (ci >= Ci) {
                ci -= Ci;
                ++t;
            }
        }
    }
    const int zz = z0 + wave;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = j * 16 + (lane & 15);
        if (co >= Co) continue;
        const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = (lane >> 4) * 4 + i;           // row of the 16-voxel tile
                const int yy = y0 + 2 * m + (r >> 3), xx = x0 + (r & 7);
                if (zz >= g.D || yy >= g.H || xx >= g.W) continue;
                const long long v = (((long long)b * g.D + zz) * g.H + yy) * g.W + xx;
                float rr = acc[m][j][i] + bb;
                if (act) rr = lrelu(rr, alpha);
                if (y16) y16[v * Co + co] = f2bf(rr);
                if (y32) y32[v * Co + co] = accumulate ? y32[v * Co + co] + rr : rr;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The halo-brick convolution with the input channel count fixed at compile
// time, for the few-channel layers with 32 outputs (Ci in {16, 32}; those
// with 16 outputs take the row-reuse kernel below): the B fragments
// (weights) of the K steps live in
// registers, read from memory in chunks of CH steps, the next chunk in
// flight while the current one feeds the matrix cores, and the whole
// 6 x 6 x 18 input brick is fetched with every load issued before the
// first LDS store, so a workgroup waits for one memory round trip before
// its matrix-core work rather than one per staging pass.  The LDS offset of
// a lane's (tap, channel) pair at K step s (k = 32 s + 8 (l / 16)) is a
// compile-time constant picked by the lane's quarter.  Consecutive
// workgroups are dealt round-robin to the 8 XCDs, so the brick order is
// permuted to give each XCD one contiguous range of bricks: neighbouring
// bricks, which share halo voxels, then meet in the same L2.
// ---------------------------------------------------------------------------
template <int CI>
__host__ __device__ constexpr int halo_elem(int k) {
    // element offset of k = t CI + ci from the output voxel's own LDS slot
    return k >= 27 * CI ? 0
                        : ((((k / CI) / 9 - 1) * (kRY + 2) + ((k / CI) / 3) % 3 - 1) * (kRX + 2) +
                           (k / CI) % 3 - 1) * (CI + 8) + k % CI;
}

constexpr int kXcds = 8;
// Below this many bricks a launch of one workgroup per brick leaves the
// device partly idle (256 CUs, two or more workgroups each), so the brick
// kernels split 64 or more output channels into groups of 32, one per
// blockIdx.y.
constexpr long long kFewBricks = 2048;

__device__ __forceinline__ int xcd_contiguous(int bid, int nblocks) {
    const int q = nblocks / kXcds, r = nblocks % kXcds;
    const int xcd = bid % kXcds, idx = bid / kXcds;
    return xcd * q + (xcd < r ? xcd : r) + idx;
}

template <int CI, int NT, int CH>
__global__ void __launch_bounds__(256) k_conv_fwd_reg(const uint16_t* __restrict__ x,
                                                      const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias, Geo g,
                                                      int Co, float alpha, int act,
                                                      uint16_t* __restrict__ y16,
                                                      float* __restrict__ y32, int accumulate,
                                                      const uint16_t* __restrict__ ym) {
    constexpr int MT = 4;
    constexpr int K = 27 * CI;
    constexpr int KS = (K + 31) / 32;
    constexpr int NCH = (KS + CH - 1) / CH;
    constexpr int ROW = CI + 8;
    constexpr int GV = CI / 8;
    extern __shared__ __align__(16) uint16_t hx[];   // [kRVox][ROW]
    const int nbx = (g.W + kRX - 1) / kRX, nby = (g.H + kRY - 1) / kRY, nbz = (g.D + kRZ - 1) / kRZ;
    int bid = xcd_contiguous(blockIdx.x, gridDim.x);
    const int bx = bid % nbx;
    bid /= nbx;
    const int by = bid % nby;
    bid /= nby;
    const int bz = bid % nbz;
    const int b = bid / nbz;
    const int x0 = bx * kRX, y0 = by * kRY, z0 = bz * kRZ;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, q = lane >> 4;
    // output channels [cg, cg + 16 NT) of Co (blockIdx.y picks the group)
    const int cg = blockIdx.y * NT * 16;
    w += (long long)cg * K;
    if (bias) bias += cg;
    if (y16) y16 += cg;
    if (y32) y32 += cg;
    if (ym) ym += cg;
    // Loads go through buffer resources with 32-bit offsets (the host keeps
    // every operand below 2 GiB); a load that must give zeros (outside the
    // volume, past the last K step) reads offset 0 and is replaced by zero,
    // so no load sits behind a branch.
    const __amdgpu_buffer_rsrc_t xr = rsrc16(x, g.nvox() * CI);
    const __amdgpu_buffer_rsrc_t wr = rsrc16(w, (long long)NT * 16 * K);
    // The weights go through LDS in chunks of CH K steps, B[k][n] = w[n][k]
    // (Co = 16 NT), each loaded once per workgroup (a 16-byte unit per
    // thread) while the previous chunk feeds the matrix cores; two buffers
    // after the brick, fragments laid out [q / 2][n][q % 2][8] (bank-disjoint
    // for the 16 lanes one clock serves).
    constexpr int NFR = CH * NT, PT = NFR * 64 / 256;
    static_assert(NFR * 64 % 256 == 0, "a chunk is whole 16-byte units per thread");
    uint16_t* wl = hx + kRVox * ROW;   // [2][NFR][512]
    auto load_chunk = [&](uint4 (&r)[PT], int c) {
#pragma unroll
        for (int e = 0; e < PT; ++e) {
            const int i = (int)threadIdx.x + 256 * e;
            const int f = i >> 6, n = (i >> 2) & 15, qq = i & 3;
            const int s2 = f / NT, j = f % NT, k = (c * CH + s2) * 32 + qq * 8;
            r[e] = ld16(wr, ((j * 16 + n) * K + k) * 2, c * CH + s2 < KS && k < K);
        }
    };
    auto store_chunk = [&](const uint4 (&r)[PT], int buf) {
#pragma unroll
        for (int e = 0; e < PT; ++e) {
            const int i = (int)threadIdx.x + 256 * e;
            const int f = i >> 6, n = (i >> 2) & 15, qq = i & 3;
            *reinterpret_cast<uint4*>(wl + (buf * NFR + f) * 512 + (qq >> 1) * 256 + n * 16 +
                                      (qq & 1) * 8) = r[e];
        }
    };
    const int wfl = (q >> 1) * 256 + (lane & 15) * 16 + (q & 1) * 8;
    uint4 wrg[PT];
    // Staging: a thread owns one 16-byte column of the halo rows (voxel hxx
    // of the row, channel group c) and walks the 6 x 6 rows RP at a time, so
    // the x part of its index and bounds test is worked out once.
    constexpr int RU = (kRX + 2) * GV;           // 16-byte units per halo row
    constexpr int NROW = (kRZ + 2) * (kRY + 2);  // halo rows
    constexpr int RP = 256 / RU;                 // rows per pass
    constexpr int NUR = (NROW + RP - 1) / RP;
    const int col = threadIdx.x % RU, r0 = threadIdx.x / RU;
    const int hxx = col / GV, c = (col - hxx * GV) * 8;
    const int xx = x0 - 1 + hxx;
    const bool xin = r0 < RP && xx >= 0 && xx < g.W;
    uint4 st[NUR];
    constexpr int kMaxR0 = 255 / RU;   // largest r0, idle threads included
    const bool inner = x0 >= 1 && x0 + kRX < g.W && y0 >= 1 && y0 + kRY < g.H && z0 >= 1 &&
                       z0 + kRZ < g.D;   // the halo lies inside the volume; uniform
    if (inner) {
        // the whole halo is inside the volume: no bounds tests, and the offset
        // advances by RP rows per pass (DZ slices and DY rows, wrapping at 6)
        constexpr int DZ = RP / (kRY + 2), DY = RP % (kRY + 2);
        const int rowb = g.W * (CI * 2), plane = g.H * rowb;
        int hyy = r0 % (kRY + 2);
        int off = (((b * g.D + z0 - 1 + r0 / (kRY + 2)) * g.H + y0 - 1 + hyy) * g.W + xx) *
                      (CI * 2) + c * 2;
#pragma unroll
        for (int u = 0; u < NUR; ++u) {
            if (kMaxR0 + RP * u < NROW) {
                st[u] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
            } else {
                const int row = r0 + RP * u;
                st[u] = ld16(xr, off, r0 < RP && row < NROW);
            }
            off += DZ * plane + DY * rowb;
            hyy += DY;
            if (hyy >= kRY + 2) {
                hyy -= kRY + 2;
                off += plane - (kRY + 2) * rowb;
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < NUR; ++u) {
            const int row = r0 + RP * u;
            const int hzz = row / (kRY + 2), hyy = row - hzz * (kRY + 2);
            const int yy = y0 - 1 + hyy, zz = z0 - 1 + hzz;
            const bool in = xin && (NROW % RP == 0 || u < NUR - 1 || row < NROW) && yy >= 0 &&
                            zz >= 0 && yy < g.H && zz < g.D;
            st[u] = ld16(xr, (((b * g.D + zz) * g.H + yy) * g.W + xx) * (CI * 2) + c * 2, in);
        }
    }
    load_chunk(wrg, 0);
#pragma unroll
    for (int u = 0; u < NUR; ++u) {
        const int row = r0 + RP * u;
        if (r0 < RP && (NROW % RP == 0 || u < NUR - 1 || row < NROW))
            *reinterpret_cast<uint4*>(hx + (row * (kRX + 2) + hxx) * ROW + c) = st[u];
    }
    store_chunk(wrg, 0);
    __syncthreads();
    // wave w owns z-slice w; row tile m is row m (16 voxels along x)
    const int base = (((wave + 1) * (kRY + 2) + 1) * (kRX + 2) + (lane & 15) + 1) * ROW;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        if (c + 1 < NCH) load_chunk(wrg, c + 1);
#pragma unroll
        for (int s2 = 0; s2 < CH; ++s2) {
            const int s = c * CH + s2;
            if (s >= KS) break;
            constexpr int kTail = K % 32;
            const int o0 = halo_elem<CI>(s * 32), o1 = halo_elem<CI>(s * 32 + 8),
                      o2 = halo_elem<CI>(s * 32 + 16), o3 = halo_elem<CI>(s * 32 + 24);
            const int o = (q & 2) ? ((q & 1) ? o3 : o2) : ((q & 1) ? o1 : o0);
            const bool kin = kTail == 0 || s < KS - 1 || q * 8 < kTail;
            bf16x8 a[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                uint4 av = *reinterpret_cast<const uint4*>(hx + base + o + m * (kRX + 2) * ROW);
                if (!kin) av = make_uint4(0, 0, 0, 0);
                a[m] = as_bf16x8(av);
            }
            bf16x8 bv[NT];
#pragma unroll
            for (int j = 0; j < NT; ++j)
                bv[j] = as_bf16x8(*reinterpret_cast<const uint4*>(
                    wl + ((c & 1) * NFR + s2 * NT + j) * 512 + wfl));
#pragma unroll
            for (int j = 0; j < NT; ++j)
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bv[j], acc[m][j], 0,
                                                                        0, 0);
        }
        // the next chunk into the other buffer, last read in the chunk before
        // this one (finished by every wave before the barrier that ended it)
        if (c + 1 < NCH) {
            store_chunk(wrg, (c + 1) & 1);
            __syncthreads();
        }
    }
    const int zz = z0 + wave;
    if (!y32) {
        // bf16 output only: the wave's 4 x 16 slice goes through LDS ([voxel][Co],
        // voxels row-major, which is the tile order) so that every lane stores
        // 16 contiguous bytes
        __syncthreads();   // every wave is done with the input brick
        uint16_t* ot = hx + wave * (64 * NT * 16);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const float bb = bias ? bias[j * 16 + (lane & 15)] : 0.0f;
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float rr = acc[m][j][i] + bb;
                    if (act) rr = lrelu(rr, alpha);
                    if (ym) {   // a LeakyReLU input gradient, as lrelu_bwd turns rr
                        const int yy = y0 + m, xx = x0 + q * 4 + i;
                        const long long v = (((long long)b * g.D + zz) * g.H + yy) * g.W + xx;
                        const float yv = zz < g.D && yy < g.H && xx < g.W
                                             ? bf2f(ym[v * Co + j * 16 + (lane & 15)])
                                             : 0.0f;
                        rr = yv > 0.0f ? rr : alpha * rr;
                    }
                    ot[(m * 16 + q * 4 + i) * (NT * 16) + j * 16 + (lane & 15)] = f2bf(rr);
                }
        }
        __syncthreads();
#pragma unroll
        for (int u0 = 0; u0 < 64 * 2 * NT; u0 += 64) {
            const int u = u0 + lane, p = u / (2 * NT), c = (u % (2 * NT)) * 8;
            const int yy = y0 + (p >> 4), xx = x0 + (p & 15);
            if (zz >= g.D || yy >= g.H || xx >= g.W) continue;
            const long long v = (((long long)b * g.D + zz) * g.H + yy) * g.W + xx;
            *reinterpret_cast<uint4*>(y16 + v * Co + c) =
                *reinterpret_cast<const uint4*>(ot + p * (NT * 16) + c);
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = j * 16 + (lane & 15);
        if (co >= Co) continue;
        const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = q * 4 + i;           // row of the 16-voxel tile
                const int yy = y0 + m, xx = x0 + r;
                if (zz >= g.D || yy >= g.H || xx >= g.W) continue;
                const long long v = (((long long)b * g.D + zz) * g.H + yy) * g.W + xx;
                float rr = acc[m][j][i] + bb;
                if (act) rr = lrelu(rr, alpha);
                if (y16) y16[v * Co + co] = f2bf(rr);
                if (y32) y32[v * Co + co] = accumulate ? y32[v * Co + co] + rr : rr;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The row-reuse convolution with 16 outputs, persistent over bricks: the
// workgroup gathers the weight fragments of every K step into registers
// once, then walks a contiguous range of this XCD's bricks (neighbouring
// bricks, which share halo voxels, run at the same time and meet in one
// L2), the next brick's input rows loaded into registers while the current
// one feeds the matrix cores.  Per brick the work is the row-reuse form of
// k_conv_fwd_reg (pairs of (dz, dx, 16-channel block) combinations, 6 input
// rows read once for 3 dy taps x 4 output rows).  The weights are the
// matrix cores' A operand and the input rows the B operand, so a lane ends
// with 4 consecutive output channels of one voxel and stores them straight
// from registers (a wave's 64 lanes write one 16-voxel row, 512 contiguous
// bytes).  Loads go through buffer resources: a halo voxel outside the
// volume is read at an offset past the end, which the hardware answers with
// zeros, so no load sits behind a branch and the compiler's wait counts stay
// exact across the loop.  With CS < CI the input is the decoder's
// concatenation, read in place: channels [0, CS) from x, [CS, CI) from the
// half-size level xl (nearest-neighbour upsampled); a thread's channel group
// comes from one of the two, the other load is answered with zeros.
// ---------------------------------------------------------------------------
constexpr int kOob = 0x7ff00000;   // a buffer offset past every operand

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Output of the row-reuse kernel: bf16 only (y16), FP32 (y32, added to when
// accumulate; y16 as well when non-null), or the network's head fused in
// (bf16 y16 when non-null, and out[v] = b + resid[v] + sum_c w[c] y[v][c]
// over the bf16-rounded outputs: each lane quarter sums its 4 channels in
// order, the quarters are added pairwise, (0 + 1) + (2 + 3)).
// Or the input gradient of a LeakyReLU layer (kOutDz): dz[v][c] =
// bf16(ym[v][c] > 0 ? r : alpha r) with r the FP32 conv output (no bias),
// what conv_fwd into FP32 followed by lrelu_bwd gives; with par non-null
// r = conv + par[p(v)][c] / 8 (p(v) the half-size parent), what pool_bwd
// with a LeakyReLU target adds and gives.  Or bf16 y16 and its
// 2 x 2 x 2 average pool (kOutPool, into pool at half size, as pool_fwd).
// Or the backward of a nearest x2 upsampling followed by a LeakyReLU
// input gradient (kOutUpDz): the FP32 conv outputs (no bias) of each
// 2 x 2 x 2 block summed, then dz[p][c] = bf16(ym[p][c] > 0 ? s : alpha s)
// at the half-size parent p (ym and dz with ys channels), with nothing
// stored at full size: what an FP32 conv output followed by up_bwd with a
// LeakyReLU target gives, up to the order of the 8-term sum.
enum { kOutBf16 = 0, kOutF32 = 1, kOutHead = 2, kOutDz = 3, kOutPool = 4, kOutUpDz = 5 };
struct HeadArgs {
    const float* w;       // [16]
    const float* b;       // [1]
    const float* resid;   // per voxel
    float* out;           // per voxel
    const uint16_t* ym;   // kOutDz: the layer's output activation, [voxel][16];
                          // kOutUpDz: the half-size activation, [parent][ys]
    uint16_t* pool;       // kOutPool: [voxel at half size][16]; kOutUpDz: dz,
                          // [parent][ys]
    const float* par;     // kOutDz: the pooled layer's gradient, [parent][16], or null
};

template <int CI, int CS, int OUT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CI == 16 ? 3 : 1)))
k_conv_rows(const uint16_t* __restrict__ x,
                                                   const uint16_t* __restrict__ xl,
                                                   const uint16_t* __restrict__ w,
                                                   const float* __restrict__ bias, Geo g,
                                                   float alpha, int act,
                                                   uint16_t* __restrict__ y16,
                                                   float* __restrict__ y32, int accumulate,
                                                   HeadArgs head, int ys) {
    constexpr bool F32 = OUT == kOutF32;
    constexpr int MT = 4, K = 27 * CI, ROW = brick_row(CI);
    constexpr int NB = CI / 16, NU = 9 * NB, NP = (NU + 1) / 2;
    constexpr int HX = kRX + 2, HY = kRY + 2, HZ = kRZ + 2;
    // Staging: a "column" is one 16-byte unit of every halo plane, fixed
    // (y, x, channel group); a thread owns columns t, t + 256, ... and loads
    // them in all HZ planes, so its per-column offsets are worked out once
    // and the planes differ by a scalar stride.  The columns of x (CS
    // channels) come first, those of xl after them.
    constexpr int GS = CS / 8, GL = (CI - CS) / 8;
    constexpr int NCS = HY * HX * GS, NCOL = NCS + HY * HX * GL;
    constexpr int NC = (NCOL + 255) / 256;
    static_assert(CI % 16 == 0 && CS % 8 == 0, "16-channel blocks");
    // [kRVox][ROW] halo brick, then one spare 16-byte slot per thread for
    // the staging stores of a thread's unused columns
    extern __shared__ __align__(16) uint16_t hx[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, q = lane >> 4;
    const int nbx = (g.W + kRX - 1) / kRX, nby = (g.H + kRY - 1) / kRY, nbz = (g.D + kRZ - 1) / kRZ;
    const int nbk = nbx * nby * nbz * g.B;   // the host keeps it below 2^31
    // output channels [16 blockIdx.y, + 16) of ys per voxel
    const int cg = blockIdx.y * 16;
    w += (long long)cg * K;
    if (bias) bias += cg;
    if (y16) y16 += cg;
    if (y32) y32 += cg;

    // the weight fragments of every pair and dy (a padded half gets zeros)
    const __amdgpu_buffer_rsrc_t wr = rsrc16(w, 16LL * K);
    bf16x8 wv[NP][3];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int u = 2 * p + (q >> 1);
        const int dz = u / (3 * NB), dx = (u / NB) % 3, cb = u % NB;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int k = (dz * 9 + dy * 3 + dx) * CI + cb * 16 + (q & 1) * 8;
            wv[p][dy] = as_bf16x8(__builtin_bit_cast(
                uint4, __builtin_amdgcn_raw_buffer_load_b128(
                           wr, u < NU ? ((lane & 15) * K + k) * 2 : kOob, 0, 0)));
        }
    }

    // per column: halo (y, x), LDS slot, byte offset from the brick's corner
    // voxel (fine for x; for xl the corner of the coarse parents)
    const int Dd = g.D >> 1, Hd = g.H >> 1, Wd = g.W >> 1;
    int cy[NC], cx[NC], lo[NC], ro[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const int col = (int)threadIdx.x + 256 * k;
        const bool used = col < NCOL, fine = col < NCS;
        const int cc = !used ? 0 : fine ? col : col - NCS, gw = fine || GL == 0 ? GS : GL;
        const int gg = cc % gw, xy = cc / gw, yv = xy / HX;
        cx[k] = xy % HX;
        cy[k] = used ? yv : -(1 << 20);   // unused columns never pass the y test
        lo[k] = used ? (xy * ROW + (fine ? 0 : CS) + gg * 8) * 2
                     : (kRVox * ROW + (int)threadIdx.x * 8) * 2;
        ro[k] = fine || !used
                    ? ((yv * g.W + cx[k]) * CS + gg * 8) * 2
                    : ((((yv + 1) >> 1) * Wd + ((cx[k] + 1) >> 1)) * (CI - CS) + gg * 8) * 2;
    }
    const __amdgpu_buffer_rsrc_t xr = rsrc16(x, g.nvox() * CS);
    const __amdgpu_buffer_rsrc_t lr = rsrc16(CS < CI ? xl : x, CS < CI ? g.nvox() / 8 * (CI - CS) : 0);
    const int planeb = g.H * g.W * CS * 2, planel = Hd * Wd * (CI - CS) * 2;

    // bricks: this XCD's contiguous range, numbered x fastest, then y within
    // a band of 4 brick rows, then z, then the band, so that the bricks in
    // flight on an XCD (about gn consecutive ones) share their x, z and most
    // y halo voxels in its L2; the coordinates advance by gn with
    // mixed-radix carries (no divisions in the loop)
    const int yt = nby % 4 == 0 ? 4 : 1, nyb = nby / yt;
    const int xcd = blockIdx.x % kXcds, gi = blockIdx.x / kXcds;
    const int gn = ((int)gridDim.x - xcd + kXcds - 1) / kXcds;
    const int per = nbk / kXcds, rem = nbk % kXcds;
    const int s0 = xcd * per + (xcd < rem ? xcd : rem), s1 = s0 + per + (xcd < rem ? 1 : 0);
    struct Bk {
        int x, yi, z, yb, b;   // brick row y = yb yt + yi
        __device__ int y(int t) const { return yb * t + yi; }
    };
    auto split = [&](int bid) {
        Bk r;
        r.x = bid % nbx;
        bid /= nbx;
        r.yi = bid % yt;
        bid /= yt;
        r.z = bid % nbz;
        bid /= nbz;
        r.yb = bid % nyb;
        r.b = bid / nyb;
        return r;
    };
    const Bk step = split(gn);
    auto advance = [&](Bk r) {
        r.x += step.x;
        int c = r.x >= nbx;
        r.x -= c ? nbx : 0;
        r.yi += step.yi + c;
        c = r.yi >= yt;
        r.yi -= c ? yt : 0;
        r.z += step.z + c;
        c = r.z >= nbz;
        r.z -= c ? nbz : 0;
        r.yb += step.yb + c;
        c = r.yb >= nyb;
        r.yb -= c ? nyb : 0;
        r.b += step.b + c;
        return r;
    };
    auto load_brick = [&](const Bk& bk, uint4 (&st)[NC][HZ]) {
        const int x0 = bk.x * kRX, y0 = bk.y(yt) * kRY, z0 = bk.z * kRZ;
        // corner voxel (x0 - 1, y0 - 1, z0 - 1) and its coarse parent's
        // corner (x0 / 2 - 1, ...): scalar, possibly negative
        const int cf = (((bk.b * g.D + z0 - 1) * g.H + y0 - 1) * g.W + x0 - 1) * (CS * 2);
        const int cl = (((bk.b * Dd + (z0 >> 1) - 1) * Hd + (y0 >> 1) - 1) * Wd + (x0 >> 1) - 1) *
                       ((CI - CS) * 2);
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int xx = x0 - 1 + cx[k], yy = y0 - 1 + cy[k];
            const bool cin = xx >= 0 && xx < g.W && yy >= 0 && yy < g.H;
            const int col0 = 256 * k;   // this pass's first column: which sources it may hold
#pragma unroll
            for (int hz = 0; hz < HZ; ++hz) {
                const int zz = z0 - 1 + hz;
                const bool in = cin && zz >= 0 && zz < g.D;
                uint4 v = make_uint4(0, 0, 0, 0);
                if (col0 < NCS) {
                    const bool f = (int)threadIdx.x + col0 < NCS;
                    v = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                                      xr, in && f ? cf + hz * planeb + ro[k] : kOob,
                                                      0, 0));
                }
                if (CS < CI && col0 + 255 >= NCS) {
                    const bool f = (int)threadIdx.x + col0 >= NCS;
                    const uint4 u = __builtin_bit_cast(
                        uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                   lr, in && f ? cl + ((hz + 1) >> 1) * planel + ro[k] : kOob, 0, 0));
                    v.x |= u.x;
                    v.y |= u.y;
                    v.z |= u.z;
                    v.w |= u.w;
                }
                st[k][hz] = v;
            }
        }
    };

    const int rbase = ((wave * HY) * HX + (lane & 15)) * ROW + (q & 1) * 8;
    float bq[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bq[i] = bias ? bias[q * 4 + i] : 0.0f;
    // r > 0 ? r : slope r is LeakyReLU(r, alpha) for any alpha, and r when act == 0
    const float slope = act ? alpha : 1.0f;
    const __amdgpu_buffer_rsrc_t yr = rsrc16(y16, y16 ? g.nvox() * ys - cg : 0);
    float hw[4] = {0.f, 0.f, 0.f, 0.f}, hb = 0.0f;
    __amdgpu_buffer_rsrc_t rr_, or_;
    __amdgpu_buffer_rsrc_t pa_;
    if constexpr (OUT == kOutDz) {
        rr_ = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(head.ym), 0,
                                                (int)(g.nvox() * 32), 0x00020000);
        pa_ = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(head.par), 0,
                                                head.par ? (int)(g.nvox() / 8 * 64) : 0,
                                                0x00020000);
    }
    if constexpr (OUT == kOutHead) {
#pragma unroll
        for (int i = 0; i < 4; ++i) hw[i] = head.w[q * 4 + i];
        hb = head.b[0];
        rr_ = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(head.resid), 0,
                                                (int)(g.nvox() * 4), 0x00020000);
        or_ = __builtin_amdgcn_make_buffer_rsrc(head.out, 0, (int)(g.nvox() * 4), 0x00020000);
    }
    // kOutPool, kOutUpDz: the block partial sums of waves 1 and 3, handed to
    // waves 0 and 2
    constexpr bool BLK = OUT == kOutPool || OUT == kOutUpDz;
    __shared__ float pex[BLK ? 2 : 1][64][8];
    const Geo gp{g.B, g.D >> 1, g.H >> 1, g.W >> 1};
    const __amdgpu_buffer_rsrc_t pr =
        rsrc16(head.pool, OUT == kOutPool && head.pool   ? gp.nvox() * 16
                          : OUT == kOutUpDz && head.pool ? gp.nvox() * ys
                                                         : 0);
    const __amdgpu_buffer_rsrc_t ur =
        rsrc16(head.ym, OUT == kOutUpDz && head.ym ? gp.nvox() * ys : 0);
    uint4 st[NC][HZ];
    int brick = s0 + gi;
    Bk cur = split(brick < s1 ? brick : 0);
    if (brick < s1) load_brick(cur, st);
    // every load so far has landed (the weights stay live across the loop;
    // without this the compiler's wait counts would assume them pending)
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    for (; brick < s1; brick += gn) {
        __syncthreads();   // the previous brick's LDS reads are done
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
            for (int hz = 0; hz < HZ; ++hz)
                *reinterpret_cast<uint4*>(reinterpret_cast<char*>(hx) + lo[k] +
                                          (NC * 256 > NCOL && 256 * k + 255 >= NCOL
                                               ? ((int)threadIdx.x + 256 * k < NCOL ? hz : 0)
                                               : hz) * (HY * HX * ROW * 2)) = st[k][hz];
        __syncthreads();
        const Bk nxt = advance(cur);
        if (brick + gn < s1) load_brick(nxt, st);   // in flight during the MFMAs
        // output voxels of this lane: (x0 + lane % 16, y0 + m, z0 + wave)
        const int xx = cur.x * kRX + (lane & 15), y0 = cur.y(yt) * kRY, zz = cur.z * kRZ + wave;
        const bool xzin = zz < g.D && xx < g.W;
        const int v0 = ((cur.b * g.D + zz) * g.H + y0) * g.W + xx;
        float res[MT];   // the head's residual input, loaded during the MFMAs
        u32x2 ymk[MT];   // kOutDz: the activation's 4 channels, loaded during the MFMAs
        // kOutUpDz: the parents this lane stores (even lanes of waves 0 and
        // 2, two y rows), their offsets and activations, loaded likewise
        int upo[2];
        u32x2 ymp[2];
        if constexpr (OUT == kOutUpDz) {
            const int px = xx >> 1, pz = zz >> 1;
#pragma unroll
            for (int mp = 0; mp < 2; ++mp) {
                const int py = (y0 >> 1) + mp;
                const bool pok = !(wave & 1) && !(lane & 1) && px < gp.W && py < gp.H && pz < gp.D;
                upo[mp] = pok ? ((((cur.b * gp.D + pz) * gp.H + py) * gp.W + px) * ys + cg + q * 4) * 2
                              : kOob;
                ymp[mp] = __builtin_amdgcn_raw_buffer_load_b64(ur, upo[mp], 0, 0);
            }
        }
        if constexpr (OUT == kOutHead) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
                res[m] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                    rr_, xzin && y0 + m < g.H ? (v0 + m * g.W) * 4 : kOob, 0, 0));
        }
        f32x4 pp[MT / 2];   // kOutDz with par: the parents' 4 channels (rows m, m + 1 share one)
        if constexpr (OUT == kOutDz) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
                ymk[m] = __builtin_amdgcn_raw_buffer_load_b64(
                    rr_, xzin && y0 + m < g.H ? ((v0 + m * g.W) * 16 + q * 4) * 2 : kOob, 0, 0);
            if (head.par) {
#pragma unroll
                for (int mp = 0; mp < MT / 2; ++mp) {
                    const int pv = ((cur.b * gp.D + (zz >> 1)) * gp.H + (y0 >> 1) + mp) * gp.W +
                                   (xx >> 1);
                    pp[mp] = __builtin_bit_cast(
                        f32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                   pa_, xzin && y0 + 2 * mp < g.H ? (pv * 16 + q * 4) * 4 : kOob,
                                   0, 0));
                }
            } else {
#pragma unroll
                for (int mp = 0; mp < MT / 2; ++mp) pp[mp] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
        }
        // the accumulators start at the bias
        f32x4 acc[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = f32x4{bq[0], bq[1], bq[2], bq[3]};
        auto pair_rows = [&](int p, bf16x8 (&a)[MT + 2]) {
            const int u0 = 2 * p, u1 = 2 * p + 1 < NU ? 2 * p + 1 : 2 * p;
            const int o0 = ((u0 / (3 * NB)) * HY * HX + (u0 / NB) % 3) * ROW + (u0 % NB) * 16;
            const int o1 = ((u1 / (3 * NB)) * HY * HX + (u1 / NB) % 3) * ROW + (u1 % NB) * 16;
            const int o = (q & 2) ? o1 : o0;
#pragma unroll
            for (int i = 0; i < MT + 2; ++i)
                a[i] = as_bf16x8(*reinterpret_cast<const uint4*>(hx + rbase + o + i * HX * ROW));
        };
        if constexpr (CI == 48) {
            // one wave per SIMD: the next pair's rows are read while the
            // current pair's MFMAs run (a scheduling barrier keeps the reads
            // early), so that no other wave is needed to cover their latency
            bf16x8 a[2][MT + 2];
            pair_rows(0, a[0]);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                if (p + 1 < NP) pair_rows(p + 1, a[(p + 1) & 1]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                    for (int m = 0; m < MT; ++m)
                        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            wv[p][dy], a[p & 1][m + dy], acc[m], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                bf16x8 a[MT + 2];
                pair_rows(p, a);
#pragma unroll
                for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                    for (int m = 0; m < MT; ++m)
                        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wv[p][dy], a[m + dy],
                                                                         acc[m], 0, 0, 0);
            }
        }
        // acc[m][i]: output channel 4 q + i of voxel (x0 + lane % 16, y0 + m, z0 + wave)
        float pc[MT][4];   // kOutPool: the stored (bf16) values as floats
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const bool in = xzin && y0 + m < g.H;
            const int v = v0 + m * g.W;
            float r[4];
            if constexpr (OUT == kOutDz) {
                const float yv[4] = {__uint_as_float(ymk[m].x << 16),
                                     __uint_as_float(ymk[m].x & 0xFFFF0000u),
                                     __uint_as_float(ymk[m].y << 16),
                                     __uint_as_float(ymk[m].y & 0xFFFF0000u)};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float t = head.par ? acc[m][i] + 0.125f * pp[m >> 1][i] : acc[m][i];
                    r[i] = yv[i] > 0.0f ? t : alpha * t;
                }
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) r[i] = acc[m][i] > 0.0f ? acc[m][i] : slope * acc[m][i];
            }
            if constexpr (OUT == kOutUpDz) {
#pragma unroll
                for (int i = 0; i < 4; ++i) pc[m][i] = r[i];
            } else if constexpr (!F32) {
                // a store past the end of the resource is dropped: no branch
                const uint32_t lo16 = pk_bf16(r[0], r[1]), hi16 = pk_bf16(r[2], r[3]);
                __builtin_amdgcn_raw_buffer_store_b64(u32x2{lo16, hi16}, yr,
                                                      in ? (v * ys + q * 4) * 2 : kOob, 0, 0);
                if constexpr (OUT == kOutPool) {
                    pc[m][0] = __uint_as_float(lo16 << 16);
                    pc[m][1] = __uint_as_float(lo16 & 0xFFFF0000u);
                    pc[m][2] = __uint_as_float(hi16 << 16);
                    pc[m][3] = __uint_as_float(hi16 & 0xFFFF0000u);
                }
                if constexpr (OUT == kOutHead) {
                    // the head on the stored (bf16) values
                    float p = hw[0] * __uint_as_float(lo16 << 16);
                    p = __builtin_fmaf(hw[1], __uint_as_float(lo16 & 0xFFFF0000u), p);
                    p = __builtin_fmaf(hw[2], __uint_as_float(hi16 << 16), p);
                    p = __builtin_fmaf(hw[3], __uint_as_float(hi16 & 0xFFFF0000u), p);
                    p += __shfl_xor(p, 16);
                    p += __shfl_xor(p, 32);
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint((hb + res[m]) + p), or_,
                                                          in && q == 0 ? v * 4 : kOob, 0, 0);
                }
            } else {
                if (!in) continue;
                if (y16) {
                    uint2 pk;
                    pk.x = (uint32_t)f2bf(r[0]) | ((uint32_t)f2bf(r[1]) << 16);
                    pk.y = (uint32_t)f2bf(r[2]) | ((uint32_t)f2bf(r[3]) << 16);
                    *reinterpret_cast<uint2*>(y16 + (long long)v * ys + q * 4) = pk;
                }
                float4* d = reinterpret_cast<float4*>(y32 + (long long)v * ys + q * 4);
                float4 o4 = make_float4(r[0], r[1], r[2], r[3]);
                if (accumulate) {
                    const float4 prev = *d;
                    o4.x += prev.x;
                    o4.y += prev.y;
                    o4.z += prev.z;
                    o4.w += prev.w;
                }
                *d = o4;
            }
        }
        if constexpr (OUT == kOutPool) {
            // children (c0 + c1) + (c2 + c3) over x pairs (lanes l, l ^ 1) and
            // y pairs (rows m, m + 1) of this z-slice; waves 1 and 3 hand
            // theirs to 0 and 2, which add them and store the pooled voxels
            float t[2][4];
#pragma unroll
            for (int mp = 0; mp < 2; ++mp)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float a0 = pc[2 * mp][i], a2 = pc[2 * mp + 1][i];
                    const float a1 = __shfl_xor(a0, 1), a3 = __shfl_xor(a2, 1);
                    t[mp][i] = (a0 + a1) + (a2 + a3);
                }
            if (wave & 1) {
#pragma unroll
                for (int mp = 0; mp < 2; ++mp)
#pragma unroll
                    for (int i = 0; i < 4; ++i) pex[wave >> 1][lane][mp * 4 + i] = t[mp][i];
            }
            __syncthreads();
            if (!(wave & 1)) {
                const int px = (cur.x * kRX + (lane & 15)) >> 1, pz = (cur.z * kRZ + wave) >> 1;
#pragma unroll
                for (int mp = 0; mp < 2; ++mp) {
                    float sv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        sv[i] = (t[mp][i] + pex[wave >> 1][lane][mp * 4 + i]) * 0.125f;
                    const int py = (y0 >> 1) + mp;
                    const bool pok = !(lane & 1) && px < gp.W && py < gp.H && pz < gp.D;
                    const int pv = ((cur.b * gp.D + pz) * gp.H + py) * gp.W + px;
                    __builtin_amdgcn_raw_buffer_store_b64(
                        u32x2{pk_bf16(sv[0], sv[1]), pk_bf16(sv[2], sv[3])}, pr,
                        pok ? (pv * 16 + q * 4) * 2 : kOob, 0, 0);
                }
            }
        }
        if constexpr (OUT == kOutUpDz) {
            // the block sums as for kOutPool (x pairs, y pairs, then z pairs
            // through LDS), unscaled, through the parent's LeakyReLU
            float t[2][4];
#pragma unroll
            for (int mp = 0; mp < 2; ++mp)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float a0 = pc[2 * mp][i], a2 = pc[2 * mp + 1][i];
                    const float a1 = __shfl_xor(a0, 1), a3 = __shfl_xor(a2, 1);
                    t[mp][i] = (a0 + a1) + (a2 + a3);
                }
            if (wave & 1) {
#pragma unroll
                for (int mp = 0; mp < 2; ++mp)
#pragma unroll
                    for (int i = 0; i < 4; ++i) pex[wave >> 1][lane][mp * 4 + i] = t[mp][i];
            }
            __syncthreads();
            if (!(wave & 1)) {
#pragma unroll
                for (int mp = 0; mp < 2; ++mp) {
                    const float yv[4] = {__uint_as_float(ymp[mp].x << 16),
                                         __uint_as_float(ymp[mp].x & 0xFFFF0000u),
                                         __uint_as_float(ymp[mp].y << 16),
                                         __uint_as_float(ymp[mp].y & 0xFFFF0000u)};
                    float dv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float sv = t[mp][i] + pex[wave >> 1][lane][mp * 4 + i];
                        dv[i] = yv[i] > 0.0f ? sv : alpha * sv;
                    }
                    __builtin_amdgcn_raw_buffer_store_b64(
                        u32x2{pk_bf16(dv[0], dv[1]), pk_bf16(dv[2], dv[3])}, pr, upo[mp], 0, 0);
                }
            }
        }
        cur = nxt;
    }
}

// ---------------------------------------------------------------------------
// The first convolution (16 outputs) from the network input's two used
// channels, normalised dose and density, packed as one 32-bit bf16 pair per
// voxel (x2[v] = bf16(d) | bf16(rho) << 16); the other input channels are
// zero and drop out of the sum.  K = 27 taps x 2 channels, k = 2 t + c,
// padded to two K steps of 32 (taps 27..31 have zero weights).  Persistent
// over 4 x 4 x 16 bricks like k_conv_rows: the weights are gathered into
// registers once, the next brick's halo (6 x 6 x 18 pairs, 2.6 KB) is
// loaded while the current one feeds the matrix cores, and a lane's input
// fragment is its 4 taps x 2 channels, read as 4 pairs from the halo.
// Weights [16][27][cin]: only channels 0 and 1 are read.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_conv_in(const uint32_t* __restrict__ x2,
                                                 const uint16_t* __restrict__ w, int cin,
                                                 const float* __restrict__ bias, Geo g,
                                                 float alpha, uint16_t* __restrict__ y16) {
    constexpr int MT = 4, HX = kRX + 2, HY = kRY + 2, HZ = kRZ + 2;
    constexpr int NH = HZ * HY * HX, NL = (NH + 255) / 256;
    __shared__ uint32_t hx[NH + 256];   // halo pairs, then a spare slot per thread
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, q = lane >> 4;
    const int nbx = (g.W + kRX - 1) / kRX, nby = (g.H + kRY - 1) / kRY, nbz = (g.D + kRZ - 1) / kRZ;
    const int nbk = nbx * nby * nbz * g.B;

    // A = W[co][k]: lane (co = lane % 16, quarter q) holds k = 32 s + 8 q + [0, 8),
    // i.e. taps 16 s + 4 q + [0, 4), two channels each, as 4 32-bit words
    const __amdgpu_buffer_rsrc_t wr = rsrc16(w, 16LL * 27 * cin);
    bf16x8 wa[2];
    int off[2][4];   // LDS word offset of each of the lane's taps from the row-0 slot
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
        uint32_t wd[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = 16 * s2 + 4 * q + i;
            wd[i] = __builtin_amdgcn_raw_buffer_load_b32(
                wr, t < 27 ? (((lane & 15) * 27 + t) * cin) * 2 : kOob, 0, 0);
            off[s2][i] = t < 27 ? ((t / 9) * HY + (t / 3) % 3) * HX + t % 3 : 0;
        }
        wa[s2] = as_bf16x8(make_uint4(wd[0], wd[1], wd[2], wd[3]));
    }
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(x2), 0, (int)(g.nvox() * 4), 0x00020000);
    const __amdgpu_buffer_rsrc_t yr = rsrc16(y16, g.nvox() * 16);
    // staging: thread t loads halo slots t, t + 256, t + 512 (< NH), at byte
    // offsets rel from the brick's corner voxel (x0 - 1, y0 - 1, z0 - 1)
    int sy[NL], sx[NL], sz[NL], rel[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int h = (int)threadIdx.x + 256 * k;
        sx[k] = h % HX;
        sy[k] = (h / HX) % HY;
        sz[k] = h < NH ? h / (HX * HY) : -(1 << 20);
        rel[k] = h < NH ? (((h / (HX * HY)) * g.H + sy[k]) * g.W + sx[k]) * 4 : 0;
    }
    struct Bk { int x, y, z, b; };
    auto split = [&](int bid) {
        Bk r;
        r.x = bid % nbx;
        bid /= nbx;
        r.y = bid % nby;
        bid /= nby;
        r.z = bid % nbz;
        r.b = bid / nbz;
        return r;
    };
    const int xcd = blockIdx.x % kXcds, gi = blockIdx.x / kXcds;
    const int gn = ((int)gridDim.x - xcd + kXcds - 1) / kXcds;
    const int per = nbk / kXcds, rem = nbk % kXcds;
    const int s0 = xcd * per + (xcd < rem ? xcd : rem), s1 = s0 + per + (xcd < rem ? 1 : 0);
    const Bk step = split(gn);
    auto advance = [&](Bk r) {
        r.x += step.x;
        int c = r.x >= nbx;
        r.x -= c ? nbx : 0;
        r.y += step.y + c;
        c = r.y >= nby;
        r.y -= c ? nby : 0;
        r.z += step.z + c;
        c = r.z >= nbz;
        r.z -= c ? nbz : 0;
        r.b += step.b + c;
        return r;
    };
    auto load_brick = [&](const Bk& bk, uint32_t (&st)[NL]) {
        const int x0 = bk.x * kRX, y0 = bk.y * kRY, z0 = bk.z * kRZ;
        const int corner = (((bk.b * g.D + z0 - 1) * g.H + y0 - 1) * g.W + x0 - 1) * 4;
        if (x0 >= 1 && x0 + kRX < g.W && y0 >= 1 && y0 + kRY < g.H && z0 >= 1 &&
            z0 + kRZ < g.D) {
            // the halo lies inside the volume (uniform): no bounds tests
#pragma unroll
            for (int k = 0; k < NL; ++k)
                st[k] = __builtin_amdgcn_raw_buffer_load_b32(
                    xr, (int)threadIdx.x + 256 * k < NH ? corner + rel[k] : kOob, 0, 0);
        } else {
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int xx = x0 - 1 + sx[k], yy = y0 - 1 + sy[k], zz = z0 - 1 + sz[k];
                const bool in = xx >= 0 && yy >= 0 && zz >= 0 && xx < g.W && yy < g.H && zz < g.D;
                st[k] = __builtin_amdgcn_raw_buffer_load_b32(xr, in ? corner + rel[k] : kOob, 0, 0);
            }
        }
    };
    float bq[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bq[i] = bias ? bias[q * 4 + i] : 0.0f;
    const int rbase = (wave * HY) * HX + (lane & 15);   // word offset of the lane's row-0 slot
    uint32_t st[NL];
    int brick = s0 + gi;
    Bk cur = split(brick < s1 ? brick : 0);
    if (brick < s1) load_brick(cur, st);
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the weights have landed
    for (; brick < s1; brick += gn) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int h = (int)threadIdx.x + 256 * k;
            hx[h < NH ? h : NH + (int)threadIdx.x] = st[k];
        }
        __syncthreads();
        const Bk nxt = advance(cur);
        if (brick + gn < s1) load_brick(nxt, st);
        f32x4 acc[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            acc[m] = f32x4{bq[0], bq[1], bq[2], bq[3]};
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                const int b0 = rbase + m * HX;
                const uint4 bv = make_uint4(hx[b0 + off[s2][0]], hx[b0 + off[s2][1]],
                                            hx[b0 + off[s2][2]], hx[b0 + off[s2][3]]);
                acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[s2], as_bf16x8(bv), acc[m], 0,
                                                                 0, 0);
            }
        }
        const int xx = cur.x * kRX + (lane & 15), y0 = cur.y * kRY, zz = cur.z * kRZ + wave;
        const bool xzin = zz < g.D && xx < g.W;
        const int v0 = ((cur.b * g.D + zz) * g.H + y0) * g.W + xx;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const bool in = xzin && y0 + m < g.H;
            float r[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) r[i] = acc[m][i] > 0.0f ? acc[m][i] : alpha * acc[m][i];
            const uint32_t lo16 = pk_bf16(r[0], r[1]), hi16 = pk_bf16(r[2], r[3]);
            __builtin_amdgcn_raw_buffer_store_b64(u32x2{lo16, hi16}, yr,
                                                  in ? ((v0 + m * g.W) * 16 + q * 4) * 2 : kOob, 0,
                                                  0);
        }
        cur = nxt;
    }
}

// ---------------------------------------------------------------------------
// The halo-brick convolution for wide inputs (Ci a multiple of 32, at least
// 64) with 32 or 64 outputs: the input channels are taken 32 at a time
// (one pass each), so the brick of one pass (6 x 6 x 18 voxels x 32
// channels, 51 KB of LDS with the slot pad) and two weight chunks leave room
// for two workgroups per CU.  Within a pass each K step is one tap over the
// pass's 32 channels, so the LDS offset of a step is the tap's, uniform over
// the wave.  The next pass's brick is fetched with every load in flight
// before the first store; the weights go through LDS in chunks of CH taps,
// each loaded once per workgroup (a 16-byte unit per thread) while the
// previous chunk feeds the matrix cores (every wave fetching every fragment
// from L2 kept the vector-memory queue full).  Channels [0, cs) come from x
// (cs per voxel) and [cs, Ci) from the half-size level xl,
// nearest-neighbour upsampled (the decoder's concatenation; cs = Ci for a
// plain input).  K order: pass, tap, channel.
// ---------------------------------------------------------------------------
template <int NT, int CH, int OCC = 2>
__global__ void __launch_bounds__(256, OCC) k_conv_fwd_pass(const uint16_t* __restrict__ x,
                                                       const uint16_t* __restrict__ xl,
                                                       const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias, Geo g,
                                                       int Ci, int cs, int Co, float alpha,
                                                       int act, uint16_t* __restrict__ y16,
                                                       float* __restrict__ y32, int accumulate,
                                                       const uint16_t* __restrict__ ym) {
    constexpr int MT = 4;
    constexpr int CP = 32;
    constexpr int ROW = CP + 8;
    constexpr int GV = CP / 8;
    constexpr int U = kRVox * GV;
    constexpr int NU = (U + 255) / 256;
    constexpr int NCH = (27 + CH - 1) / CH;
    static_assert(NCH % 2 == 0, "every pass must start on weight buffer 0");
    extern __shared__ __align__(16) uint16_t hx[];   // [kRVox][ROW]
    const int nbx = (g.W + kRX - 1) / kRX, nby = (g.H + kRY - 1) / kRY, nbz = (g.D + kRZ - 1) / kRZ;
    int bid = xcd_contiguous(blockIdx.x, gridDim.x);
    const int bx = bid % nbx;
    bid /= nbx;
    const int by = bid % nby;
    bid /= nby;
    const int bz = bid % nbz;
    const int b = bid / nbz;
    const int x0 = bx * kRX, y0 = by * kRY, z0 = bz * kRZ;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, q = lane >> 4;
    const int K = 27 * Ci, P = Ci / CP, cu = Ci - cs;
    // output channels [cg, cg + 16 NT) of Co (blockIdx.y picks the group)
    const int cg = blockIdx.y * NT * 16;
    w += (long long)cg * K;
    if (bias) bias += cg;
    if (y16) y16 += cg;
    if (y32) y32 += cg;
    if (ym) ym += cg;
    auto load_brick = [&](uint4 (&st)[NU], int p) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int i = threadIdx.x + u * 256;
            st[u] = make_uint4(0, 0, 0, 0);
            if (i < U) {
                const int hv = i / GV, c = p * CP + (i - hv * GV) * 8;
                const int hxx = hv % (kRX + 2), hyy = (hv / (kRX + 2)) % (kRY + 2),
                          hzz = hv / ((kRX + 2) * (kRY + 2));
                const int xx = x0 - 1 + hxx, yy = y0 - 1 + hyy, zz = z0 - 1 + hzz;
                if (xx >= 0 && yy >= 0 && zz >= 0 && xx < g.W && yy < g.H && zz < g.D) {
                    if (c < cs) {
                        const long long v = (((long long)b * g.D + zz) * g.H + yy) * g.W + xx;
                        st[u] = *reinterpret_cast<const uint4*>(x + v * cs + c);
                    } else {
                        const long long v =
                            (((long long)b * (g.D >> 1) + (zz >> 1)) * (g.H >> 1) + (yy >> 1)) *
                                (g.W >> 1) + (xx >> 1);
                        st[u] = *reinterpret_cast<const uint4*>(xl + v * cu + (c - cs));
                    }
                }
            }
        }
    };
    auto store_brick = [&](const uint4 (&st)[NU]) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int i = threadIdx.x + u * 256;
            if (i < U) {
                const int hv = i / GV, c = (i - hv * GV) * 8;
                *reinterpret_cast<uint4*>(hx + hv * ROW + c) = st[u];
            }
        }
    };
    // chunk c of pass p: taps [c CH, c CH + CH) over channels [p CP, p CP + CP),
    // staged once per workgroup in LDS (two buffers: the next chunk is loaded
    // while the current one feeds the matrix cores) instead of every wave
    // fetching all of it.  A chunk is CH NT fragments B[k][n] = w[n][k] of
    // 16 outputs x 32 channels; in LDS a fragment is [q / 2][n][q % 2][8]
    // (q the lane quarter, 8 channels each), so that the 16 lanes one clock
    // serves (8 of one quarter, 8 of the next) read 16 distinct bank groups.
    constexpr int NFR = CH * NT;                // fragments per chunk
    constexpr int PT = NFR * 64 / 256;          // 16-byte units per thread and chunk
    static_assert(NFR * 64 % 256 == 0, "a chunk is whole 16-byte units per thread");
    uint16_t* wl = hx + kRVox * ROW;            // [2][NFR][512] after the brick
    const __amdgpu_buffer_rsrc_t wres =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(w), 0, Co * K * 2, 0x00020000);
    auto load_chunk = [&](uint4 (&r)[PT], int p, int c) {
#pragma unroll
        for (int e = 0; e < PT; ++e) {
            const int i = (int)threadIdx.x + 256 * e;   // 16-byte unit of the chunk
            const int f = i >> 6, n = (i >> 2) & 15, qq = i & 3;
            const int s2 = f / NT, j = f % NT, t = c * CH + s2;
            r[e] = make_uint4(0, 0, 0, 0);
            if (t < 27)
                r[e] = __builtin_bit_cast(
                    uint4, __builtin_amdgcn_raw_buffer_load_b128(
                               wres, ((j * 16 + n) * K + t * Ci + p * CP + qq * 8) * 2, 0, 0));
        }
    };
    auto store_chunk = [&](const uint4 (&r)[PT], int buf) {
#pragma unroll
        for (int e = 0; e < PT; ++e) {
            const int i = (int)threadIdx.x + 256 * e;
            const int f = i >> 6, n = (i >> 2) & 15, qq = i & 3;
            *reinterpret_cast<uint4*>(wl + (buf * NFR + f) * 512 + (qq >> 1) * 256 + n * 16 +
                                      (qq & 1) * 8) = r[e];
        }
    };
    // the lane's element offset within a fragment
    const int wfl = (q >> 1) * 256 + (lane & 15) * 16 + (q & 1) * 8;
    uint4 wr[PT];
    uint4 st[NU];
    load_brick(st, 0);
    load_chunk(wr, 0, 0);
    store_brick(st);
    store_chunk(wr, 0);
    __syncthreads();
    const int base = (((wave + 1) * (kRY + 2) + 1) * (kRX + 2) + (lane & 15) + 1) * ROW + q * 8;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const bool more = c + 1 < NCH || p + 1 < P;
            if (c + 1 < NCH) load_chunk(wr, p, c + 1);
            else if (p + 1 < P) load_chunk(wr, p + 1, 0);
#pragma unroll
            for (int s2 = 0; s2 < CH; ++s2) {
                const int t = c * CH + s2;
                if (t >= 27) break;
                const int off = ((t / 9 - 1) * (kRY + 2) + (t / 3) % 3 - 1) * (kRX + 2) + t % 3 - 1;
                bf16x8 a[MT], bv[NT];
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    a[m] = as_bf16x8(*reinterpret_cast<const uint4*>(
                        hx + base + off * ROW + m * (kRX + 2) * ROW));
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    bv[j] = as_bf16x8(*reinterpret_cast<const uint4*>(
                        wl + ((c & 1) * NFR + s2 * NT + j) * 512 + wfl));
#pragma unroll
                for (int j = 0; j < NT; ++j)
#pragma unroll
                    for (int m = 0; m < MT; ++m)
                        acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bv[j],
                                                                            acc[m][j], 0, 0, 0);
            }
            // the next chunk into the other buffer (last read in the chunk
            // before this one, which every wave finished before the barrier
            // that ended it)
            if (more) store_chunk(wr, (c + 1) & 1);
            __syncthreads();
        }
        if (p + 1 < P) {
            load_brick(st, p + 1);
            store_brick(st);
            __syncthreads();
        }
    }
    const int zz = z0 + wave;
    if (!y32) {
        // bf16 output only: stage the wave's 4 x 16 slice in LDS, 16-byte stores
        uint16_t* ot = hx + wave * (64 * NT * 16);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const float bb = bias ? bias[j * 16 + (lane & 15)] : 0.0f;
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float rr = acc[m][j][i] + bb;
                    if (act) rr = lrelu(rr, alpha);
                    if (ym) {   // a LeakyReLU input gradient, as lrelu_bwd turns rr
                        const int yy = y0 + m, xx = x0 + q * 4 + i;
                        const long long v = (((long long)b * g.D + zz) * g.H + yy) * g.W + xx;
                        const float yv = zz < g.D && yy < g.H && xx < g.W
                                             ? bf2f(ym[v * Co + j * 16 + (lane & 15)])
                                             : 0.0f;
                        rr = yv > 0.0f ? rr : alpha * rr;
                    }
                    ot[(m * 16 + q * 4 + i) * (NT * 16) + j * 16 + (lane & 15)] = f2bf(rr);
                }
        }
        __syncthreads();
#pragma unroll
        for (int u0 = 0; u0 < 64 * 2 * NT; u0 += 64) {
            const int u = u0 + lane, p = u / (2 * NT), c = (u % (2 * NT)) * 8;
            const int yy = y0 + (p >> 4), xx = x0 + (p & 15);
            if (zz >= g.D || yy >= g.H || xx >= g.W) continue;
            const long long v = (((long long)b * g.D + zz) * g.H + yy) * g.W + xx;
            *reinterpret_cast<uint4*>(y16 + v * Co + c) =
                *reinterpret_cast<const uint4*>(ot + p * (NT * 16) + c);
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = j * 16 + (lane & 15);
        const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = q * 4 + i;
                const int yy = y0 + m, xx = x0 + r;
                if (zz >= g.D || yy >= g.H || xx >= g.W) continue;
                const long long v = (((long long)b * g.D + zz) * g.H + yy) * g.W + xx;
                float rr = acc[m][j][i] + bb;
                if (act) rr = lrelu(rr, alpha);
                if (y16) y16[v * Co + co] = f2bf(rr);
                y32[v * Co + co] = accumulate ? y32[v * Co + co] + rr : rr;
            }
        }
    }
}

// LDS of k_conv_fwd_pass<NT, CH>: the brick of one pass, then two weight
// chunks of CH NT 1 KB fragments.
constexpr size_t pass_lds_bytes(int nt, int ch) {
    return ((size_t)kRVox * 40 + 2 * (size_t)nt * ch * 512) * sizeof(uint16_t);
}

// wt[ci][26 - t][co] = w[co][t][ci]: the weights of the input-gradient conv.
__global__ void k_flip_transpose(const uint16_t* w, uint16_t* wt, int Ci, int Co) {
    const int n = Co * 27 * Ci;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int ci = i % Ci, t = (i / Ci) % 27, co = i / (27 * Ci);
        wt[((size_t)ci * 27 + (26 - t)) * Co + co] = w[i];
    }
}

// ---------------------------------------------------------------------------
// Weight and bias gradients, split over voxel chunks:
//   part[c][t][co][ci] = sum_{v in chunk c} dz[v][co] x[shift(v, t)][ci],
//   part_b[c][co]      = sum_{v in chunk c} dz[v][co].
// Workgroup = (chunk, group of tg taps).  64-voxel slices of dz and of the
// tg shifted copies of x are staged transposed in LDS ([channel][voxel],
// rows padded to 72 elements = an odd number of 16-byte units, so the 16
// rows a quarter-wave reads fall on distinct banks); the dz slice is staged
// once for all taps of the group and the slice's voxel coordinates are
// decoded once.  The transpose is done in registers, 8 voxels x 8 channels
// per thread (8 16-byte loads in, 8 16-byte LDS stores out).  The block's
// tg x (Co/16) x (Ci/16) output tiles (at most 64) are spread over its 4
// waves; each lane reads 8 consecutive voxels in one 16-byte load per
// operand.
// ---------------------------------------------------------------------------
// out[c] = bf16 column c of in (8 rows of 8 bf16): element (r, c) -> (c, r)
__device__ __forceinline__ void transpose8x8(const uint4 (&in)[8], uint4 (&out)[8]) {
    uint32_t a[8][4], b[8][4];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        a[r][0] = in[r].x;
        a[r][1] = in[r].y;
        a[r][2] = in[r].z;
        a[r][3] = in[r].w;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t lo = a[2 * j][c >> 1], hi = a[2 * j + 1][c >> 1];
            b[c][j] = (c & 1) ? ((lo >> 16) | (hi & 0xFFFF0000u)) : ((lo & 0xFFFFu) | (hi << 16));
        }
#pragma unroll
    for (int c = 0; c < 8; ++c) out[c] = make_uint4(b[c][0], b[c][1], b[c][2], b[c][3]);
}

constexpr int kWgSlice = 64;
constexpr int kWgRow = kWgSlice + 8;
constexpr int kWgWaves = 4;
constexpr int kWgMaxTiles = 16;          // per wave
constexpr int kWgLdsMax = 65536;         // bytes of LDS per workgroup

int wgrad_taps_per_group(int Ci, int Co) {
    const int ntiles = (Co / 16) * (Ci / 16);
    int tg = (kWgWaves * kWgMaxTiles) / ntiles;
    if (tg > 27) tg = 27;
    if (tg < 1) tg = 1;
    while (tg > 1 && (size_t)(Co + tg * Ci) * kWgRow * sizeof(uint16_t) > (size_t)kWgLdsMax) --tg;
    return tg;
}

__global__ void __launch_bounds__(256) k_wgrad_partial(const uint16_t* __restrict__ dz,
                                                       const uint16_t* __restrict__ x, Geo g,
                                                       int Ci, int Co, int chunk, int tg,
                                                       float* __restrict__ part,
                                                       float* __restrict__ part_b) {
    extern __shared__ __align__(16) uint16_t lds[];   // [Co][kWgRow], then [tg][Ci][kWgRow]
    __shared__ int cx[kWgSlice], cy[kWgSlice], cz[kWgSlice];
    uint16_t* dzT = lds;
    uint16_t* xT = lds + Co * kWgRow;
    const int t0 = blockIdx.y * tg;
    const int ntap = min(tg, 27 - t0);
    const long long c = blockIdx.x;
    const long long v0 = c * chunk;
    const long long nv = g.nvox();
    const long long v1 = v0 + chunk < nv ? v0 + chunk : nv;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tci = Ci / 16, ntiles = (Co / 16) * tci, total = ntap * ntiles;
    const bool do_bias = blockIdx.y == 0 && tid < Co;
    const long long plane = (long long)g.W * g.H;
    f32x4 acc[kWgMaxTiles];
#pragma unroll
    for (int j = 0; j < kWgMaxTiles; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    for (long long s0 = v0; s0 < v1; s0 += kWgSlice) {
        __syncthreads();
        if (tid < kWgSlice) {
            const long long v = s0 + tid;
            if (v < v1) {
                cx[tid] = (int)(v % g.W);
                cy[tid] = (int)((v / g.W) % g.H);
                cz[tid] = (int)((v / plane) % g.D);
            } else {
                cx[tid] = -4;   // every shift leaves the volume
                cy[tid] = -4;
                cz[tid] = -4;
            }
        }
        // dz slice: an item is 8 voxels x 8 channels, loaded as 8 16-byte
        // rows, transposed in registers and stored as 8 16-byte rows
        const int gco = Co / 8, gci = Ci / 8;
        for (int i = tid; i < (kWgSlice / 8) * gco; i += blockDim.x) {
            const int vb = (i / gco) * 8, ch = (i % gco) * 8;
            uint4 in[8], out[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const long long v = s0 + vb + r;
                in[r] = v < v1 ? *reinterpret_cast<const uint4*>(dz + v * Co + ch)
                               : make_uint4(0, 0, 0, 0);
            }
            transpose8x8(in, out);
#pragma unroll
            for (int c = 0; c < 8; ++c)
                *reinterpret_cast<uint4*>(dzT + (ch + c) * kWgRow + vb) = out[c];
        }
        __syncthreads();
        // shifted x slices of the group's taps, the same 8 x 8 items
        for (int i = tid; i < ntap * (kWgSlice / 8) * gci; i += blockDim.x) {
            const int tl = i / ((kWgSlice / 8) * gci);
            const int r8 = i - tl * ((kWgSlice / 8) * gci);
            const int vb = (r8 / gci) * 8, ch = (r8 % gci) * 8;
            const int t = t0 + tl;
            const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dzz = t / 9 - 1;
            const long long shift = dx + (long long)dy * g.W + dzz * plane;
            uint4 in[8], out[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int vv = vb + r;
                const int xs = cx[vv] + dx, ys = cy[vv] + dy, zs = cz[vv] + dzz;
                in[r] = make_uint4(0, 0, 0, 0);
                if (xs >= 0 && ys >= 0 && zs >= 0 && xs < g.W && ys < g.H && zs < g.D)
                    in[r] = *reinterpret_cast<const uint4*>(x + (s0 + vv + shift) * Ci + ch);
            }
            transpose8x8(in, out);
#pragma unroll
            for (int c = 0; c < 8; ++c)
                *reinterpret_cast<uint4*>(xT + (tl * Ci + ch + c) * kWgRow + vb) = out[c];
        }
        if (do_bias)
            for (int vv = 0; vv < kWgSlice; ++vv) bsum += bf2f(dzT[tid * kWgRow + vv]);
        __syncthreads();
        const int koff = (lane >> 4) * 8;
#pragma unroll
        for (int j = 0; j < kWgMaxTiles; ++j) {
            const int tile = wave + j * kWgWaves;
            if (tile >= total) break;
            const int tl = tile / ntiles, r = tile - tl * ntiles;
            const int co0 = (r / tci) * 16, ci0 = (r % tci) * 16;
#pragma unroll
            for (int kh = 0; kh < kWgSlice; kh += 32) {
                const uint4 av = *reinterpret_cast<const uint4*>(
                    dzT + (co0 + (lane & 15)) * kWgRow + kh + koff);
                const uint4 bv = *reinterpret_cast<const uint4*>(
                    xT + (tl * Ci + ci0 + (lane & 15)) * kWgRow + kh + koff);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(av), as_bf16x8(bv),
                                                                 acc[j], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kWgMaxTiles; ++j) {
        const int tile = wave + j * kWgWaves;
        if (tile >= total) break;
        const int tl = tile / ntiles, r = tile - tl * ntiles;
        const int co0 = (r / tci) * 16, ci0 = (r % tci) * 16;
        float* out = part + ((size_t)c * 27 + t0 + tl) * Co * Ci;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            out[(size_t)(co0 + (lane >> 4) * 4 + i) * Ci + ci0 + (lane & 15)] = acc[j][i];
    }
    if (do_bias) part_b[c * Co + tid] = bsum;
}

// ---------------------------------------------------------------------------
// Weight and bias gradients of the layers with 16 or 32 outputs, by bricks:
// the same partial sums part[c][t][co][ci] as k_wgrad_partial, with chunk c
// a run of 4 x 4 x 16 voxel bricks (the bricks of k_conv_fwd_reg) and one
// workgroup per (chunk, 16 input channels).  Per brick the dz values are
// staged transposed in LDS ([co][voxel]) and the input brick with its halo
// is staged once, transposed, in three copies shifted by dx = -1, 0, +1
// ([dx][ci][6 x 6 rows][16]); every tap (dz, dy, dx) then reads aligned
// 16-byte runs of 8 voxels from copy dx at rows shifted by (dz, dy), where
// k_wgrad_partial stages a shifted copy per tap.  The dz fragments (A
// operand) of the brick's 8 K-steps stay in registers for all taps; wave w
// owns taps w, w + 4, ...  Transposes go through registers (8 x 8 bf16 per
// thread).  Row pads keep the 16 rows a quarter-wave reads on distinct
// banks.
// ---------------------------------------------------------------------------
// Row pads: a 16-byte fragment read is served 16 lanes a clock (8 lanes of
// one lane quarter with the 8 of the next), and those lanes' rows then fall
// on 16 distinct 16-byte bank groups when rows are 32, 96, 160 or 224 bytes
// apart modulo 256 (gfx950's 64 banks of 4 bytes).
constexpr int kWbXRow = 36 * 16 + 16;   // per input channel: 6 x 6 halo rows of 16 (1184 B)
constexpr int kWbDRow = 256 + 16;       // per output channel: the brick's voxels (544 B)
constexpr int kWbTaps = 7;             // taps per wave: w, w + 4, ..., < 27

int wgrad_brick_lds_bytes(int Co) { return (3 * 16 * kWbXRow + Co * kWbDRow) * 2; }

template <int NCO>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_wgrad_brick(const uint16_t* __restrict__ dz,
                                                     const uint16_t* __restrict__ x,
                                                     const uint16_t* __restrict__ xl, Geo g, int Ci,
                                                     int Cs, int bpc, int nbk,
                                                     float* __restrict__ part,
                                                     float* __restrict__ part_b, int dzc) {
    // dz: Co = 16 NCO output channels of dzc per voxel (a group of a wider layer).
    // Input channels [0, Cs) come from x (Cs per voxel), [Cs, Ci) from the
    // half-size level xl, nearest-neighbour upsampled (the decoder's
    // concatenation read in place; Cs = Ci for a plain input).
    constexpr int Co = NCO * 16;
    extern __shared__ __align__(16) uint16_t lds[];
    uint16_t* xT = lds;                          // [3][16][kWbXRow]
    uint16_t* dzT = lds + 3 * 16 * kWbXRow;      // [Co][kWbDRow]
    __shared__ float bred[256];
    const int c = blockIdx.x, ci0 = blockIdx.y * 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4;
    const int nbx = (g.W + kRX - 1) / kRX, nby = (g.H + kRY - 1) / kRY, nbz = (g.D + kRZ - 1) / kRZ;
    f32x4 acc[kWbTaps][NCO];
#pragma unroll
    for (int i = 0; i < kWbTaps; ++i)
#pragma unroll
        for (int j = 0; j < NCO; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    const int bk1 = min(nbk, (c + 1) * bpc);
    // Staging items: dz item i < 32 Co / 8 (8 voxels along x x 8 channels,
    // 8 16-byte loads) and input item i < 36 x 4 (halo row, half, channel
    // group: the 10 voxels x0 + 8 half - 1 + [0, 10), 10 loads, from which
    // the three copies shifted by dx = -1, 0, +1 take 8 each), transposed
    // into LDS.  Thread t owns dz item t and input item t; with 16 outputs
    // the next brick's loads are issued into registers before the current
    // brick's matrix-core work.
    constexpr int NDZ = 32 * (Co / 8), NXI = 36 * 4;
    uint4 rdz[8], rx[10];
    // buffer loads (32-bit offsets; the host keeps both operands below 2 GiB):
    // a voxel outside the volume is read at an offset past the end, which
    // the hardware answers with zeros, so no load sits behind a branch
    const __amdgpu_buffer_rsrc_t dzr = rsrc16(dz, g.nvox() * dzc);
    // this workgroup's 16 input channels come from one source (Cs is a
    // multiple of 16)
    const bool lowsrc = ci0 >= Cs;
    const int Cu = Ci - Cs, Dd = g.D >> 1, Hd = g.H >> 1, Wd = g.W >> 1;
    const __amdgpu_buffer_rsrc_t xr =
        lowsrc ? rsrc16(xl, (long long)Dd * Hd * Wd * g.B * Cu) : rsrc16(x, g.nvox() * Cs);
    auto load_raw = [&](int bk) {
        int r = bk;
        const int x0 = (r % nbx) * kRX;
        r /= nbx;
        const int y0 = (r % nby) * kRY;
        r /= nby;
        const int z0 = (r % nbz) * kRZ;
        const int b = r / nbz;
        {
            const int i = tid;
            const int vg = i / (Co / 8), ch = (i % (Co / 8)) * 8;
            const int rr = vg >> 1, zz = z0 + (rr >> 2), yy = y0 + (rr & 3), xs = x0 + (vg & 1) * 8;
            const bool rin = i < NDZ && zz < g.D && yy < g.H;
            const int o = ((((b * g.D + zz) * g.H + yy) * g.W + xs) * dzc + ch) * 2;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                rdz[k] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                                       dzr, rin && xs + k < g.W ? o + k * dzc * 2 : kOob,
                                                       0, 0));
        }
        {
            const int i = tid;
            const int row = i >> 2, hh = (i >> 1) & 1, cg = i & 1;
            const int zz = z0 - 1 + row / 6, yy = y0 - 1 + row % 6, xs = x0 - 1 + hh * 8;
            const bool rin = i < NXI && zz >= 0 && yy >= 0 && zz < g.D && yy < g.H;
            // voxel offset of (xs, yy, zz) and channel offset, in x or (the
            // parent voxels) in xl
            const int ov = lowsrc ? ((b * Dd + (zz >> 1)) * Hd + (yy >> 1)) * Wd
                                  : ((b * g.D + zz) * g.H + yy) * g.W + xs;
            const int oc = lowsrc ? ci0 - Cs + cg * 8 : ci0 + cg * 8;
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                const int o = lowsrc ? ((ov + ((xs + k) >> 1)) * Cu + oc) * 2 : ((ov + k) * Cs + oc) * 2;
                rx[k] = __builtin_bit_cast(
                    uint4, __builtin_amdgcn_raw_buffer_load_b128(
                               xr, rin && xs + k >= 0 && xs + k < g.W ? o : kOob, 0, 0));
            }
        }
    };
    auto store_lds = [&]() {
        uint4 out[8];
        if (tid < NDZ) {
            const int vg = tid / (Co / 8), ch = (tid % (Co / 8)) * 8;
            transpose8x8(rdz, out);
#pragma unroll
            for (int cc = 0; cc < 8; ++cc)
                *reinterpret_cast<uint4*>(dzT + (ch + cc) * kWbDRow + vg * 8) = out[cc];
        }
        if (tid < NXI) {
            const int row = tid >> 2, hh = (tid >> 1) & 1, cg = tid & 1;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                uint4 in8[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) in8[k] = rx[d + k];
                transpose8x8(in8, out);
#pragma unroll
                for (int cc = 0; cc < 8; ++cc)
                    *reinterpret_cast<uint4*>(xT + (d * 16 + cg * 8 + cc) * kWbXRow + row * 16 +
                                              hh * 8) = out[cc];
            }
        }
    };
    // 32 outputs: the registers of a prefetch would cost half the
    // occupancy, so the brick is loaded just before it is staged
    constexpr bool PF = NCO == 1;
    if (PF && c * bpc < bk1) load_raw(c * bpc);
    for (int bk = c * bpc; bk < bk1; ++bk) {
        if (!PF) load_raw(bk);
        __syncthreads();   // the previous brick's LDS reads are done
        store_lds();
        __syncthreads();
        if (PF && bk + 1 < bk1) load_raw(bk + 1);   // in flight during the MFMAs
        if (blockIdx.y == 0) {   // bias: thread (co = tid % Co) sums voxels tid / Co + k (256 / Co)
#pragma unroll 4
            for (int v = tid / Co; v < 256; v += 256 / Co) bsum += bf2f(dzT[(tid % Co) * kWbDRow + v]);
        }
        bf16x8 a[NCO][8];   // A[m = co][k = voxel] of the brick's 8 K-steps
#pragma unroll
        for (int j = 0; j < NCO; ++j)
#pragma unroll
            for (int s = 0; s < 8; ++s)
                a[j][s] = as_bf16x8(*reinterpret_cast<const uint4*>(
                    dzT + (j * 16 + (lane & 15)) * kWbDRow + s * 32 + q * 8));
#pragma unroll
        for (int i = 0; i < kWbTaps; ++i) {
            const int t = wave + 4 * i;
            if (t >= 27) break;
            const int tx = t % 3, ty = (t / 3) % 3, tz = t / 9;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                // voxels 32 s + 8 q + [0, 8): brick row 2 s + q / 2, x from 8 (q % 2)
                const int rr = 2 * s + (q >> 1);
                const int hrow = ((rr >> 2) + tz) * 6 + (rr & 3) + ty;
                const bf16x8 bv = as_bf16x8(*reinterpret_cast<const uint4*>(
                    xT + (tx * 16 + (lane & 15)) * kWbXRow + hrow * 16 + (q & 1) * 8));
#pragma unroll
                for (int j = 0; j < NCO; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j][s], bv, acc[i][j], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kWbTaps; ++i) {
        const int t = wave + 4 * i;
        if (t >= 27) break;
        float* out = part + ((size_t)c * 27 + t) * Co * Ci;
#pragma unroll
        for (int j = 0; j < NCO; ++j)
#pragma unroll
            for (int ii = 0; ii < 4; ++ii)
                out[(size_t)(j * 16 + q * 4 + ii) * Ci + ci0 + (lane & 15)] = acc[i][j][ii];
    }
    if (blockIdx.y == 0) {   // fixed-order sum of the 256 / Co partial bias sums per channel
        bred[tid] = bsum;
        __syncthreads();
        if (tid < Co) {
            float sum = 0.0f;
            for (int p = 0; p < 256 / Co; ++p) sum += bred[p * Co + tid];
            part_b[(size_t)c * Co + tid] = sum;
        }
    }
}

// dW[co][t][ci] = sum_c part[c][t][co][ci] (fixed order: deterministic).
// Deterministic column sums out[c] = sum_r part[r * ncol + c]: a workgroup
// of 64 x 16 threads owns 64 consecutive columns; row-group g sums rows
// g, g + 16, ... (coalesced across the 64 columns) and the 16 partial sums
// are added in a fixed order.  With ci_co > 0 the columns are the weight
// gradient (t, co, ci) and are written to dW[co][t][ci] (ci_co = Ci * 65536 + Co).
__global__ void __launch_bounds__(1024) k_colsum(const float* part, int nrow, int ncol,
                                                 float* out, int ci_co) {
    __shared__ float red[16][64];
    const int o = threadIdx.x & 63, gr = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + o;
    float s = 0.0f;
    if (c < ncol)
        for (int r = gr; r < nrow; r += 16) s += part[(size_t)r * ncol + c];
    red[gr][o] = s;
    __syncthreads();
    if (gr == 0 && c < ncol) {
        float t = 0.0f;
#pragma unroll
        for (int k = 0; k < 16; ++k) t += red[k][o];
        if (ci_co > 0) {
            const int Ci = ci_co >> 16, Co = ci_co & 0xFFFF;
            const int ci = c % Ci, co = (c / Ci) % Co, tap = c / (Ci * Co);
            out[((size_t)co * 27 + tap) * Ci + ci] = t;
        } else {
            out[c] = t;
        }
    }
}

// The weight and bias gradients' column sums in one launch: workgroups
// [0, nbw) sum the weight partials (columns (t, co, ci), written to
// dW[co][t][ci]), the rest the bias partials; each column in a fixed order.
__global__ void __launch_bounds__(1024) k_colsum_wb(const float* part, const float* part_b,
                                                    int nrow, int ncol, int nbw, int Co, float* dw,
                                                    float* db, int ci_co) {
    // a workgroup: 64 columns x 16 row groups (row group g sums rows g,
    // g + 16, ...), the 16 partial sums then added in a fixed order.  The
    // layer's Co outputs come in groups of cg = ci_co & 0xFFFF (each group's
    // partials [row][t][co][ci] and bias partials [row][co] one after the
    // other); column c < ncol = 27 Co Ci is (group, t, co, ci).
    __shared__ float red[16][64];
    const bool wpart = (int)blockIdx.x < nbw;
    const int Ci = ci_co >> 16, cg = ci_co & 0xFFFF;
    const int o = threadIdx.x & 63, gr = threadIdx.x >> 6;
    const int c = (wpart ? (int)blockIdx.x : (int)blockIdx.x - nbw) * 64 + o;
    const int nc = wpart ? ncol : Co;
    const int ng = 27 * cg * Ci;   // weight columns per group
    const int grp = wpart ? c / ng : c / cg, cc = wpart ? c - grp * ng : c - grp * cg;
    const float* src = wpart ? part + (size_t)grp * nrow * ng : part_b + (size_t)grp * nrow * cg;
    const int stride = wpart ? ng : cg;
    float s = 0.0f;
    if (c < nc)
        for (int r = gr; r < nrow; r += 16) s += src[(size_t)r * stride + cc];
    red[gr][o] = s;
    __syncthreads();
    if (gr == 0 && c < nc) {
        float t = 0.0f;
#pragma unroll
        for (int k = 0; k < 16; ++k) t += red[k][o];
        if (wpart) {
            const int ci = cc % Ci, co = grp * cg + (cc / Ci) % cg, tap = cc / (Ci * cg);
            dw[((size_t)co * 27 + tap) * Ci + ci] = t;
        } else {
            db[c] = t;
        }
    }
}

// dz = dy * (y > 0 ? 1 : alpha), in bf16 (LeakyReLU backward from the output sign).
__global__ void k_lrelu_bwd(const float* dy, const uint16_t* y, float alpha, long long n,
                            uint16_t* dz) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const float yy = bf2f(y[i]);
        dz[i] = f2bf(yy > 0.0f ? dy[i] : alpha * dy[i]);
    }
}

// Layout kernels.  Launched on a (ceil(W*G/256), H, D*B) grid over a
// volume's voxels: the x dimension enumerates (x, group) with G channel
// groups per voxel (8 bf16 or 4 FP32 channels per group, one 16-byte
// access), y and z come from the block index, so no thread divides by a
// runtime size except the small G.
struct VoxG {
    int x, grp;
    long long v;   // linear voxel index
    int y, z, b;
};

__device__ __forceinline__ bool vox_of(const Geo& g, int G, VoxG& o) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.W * G) return false;
    o.x = i / G;
    o.grp = i - o.x * G;
    o.y = blockIdx.y;
    o.b = blockIdx.z / g.D;
    o.z = blockIdx.z - o.b * g.D;
    o.v = ((long long)blockIdx.z * g.H + o.y) * g.W + o.x;
    return true;
}

inline dim3 vox_grid(const Geo& g, int G) {
    return dim3((unsigned)((g.W * G + 255) / 256), (unsigned)g.H, (unsigned)(g.D * g.B));
}

__device__ __forceinline__ long long child(const Geo& gc, const VoxG& c, int d) {
    // fine voxel d (0..7) of coarse voxel c; fine dims are twice gc's
    const int Wf = gc.W * 2, Hf = gc.H * 2, Df = gc.D * 2;
    return (((long long)c.b * Df + 2 * c.z + (d >> 2)) * Hf + 2 * c.y + ((d >> 1) & 1)) * Wf +
           2 * c.x + (d & 1);
}

__device__ __forceinline__ long long parent(const Geo& gf, const VoxG& f) {
    return (((long long)f.b * (gf.D / 2) + f.z / 2) * (gf.H / 2) + f.y / 2) * (gf.W / 2) + f.x / 2;
}

__device__ __forceinline__ void bf16x8_to_f32(uint4 u, float* f) {
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        f[2 * k] = __uint_as_float(w[k] << 16);
        f[2 * k + 1] = __uint_as_float(w[k] & 0xFFFF0000u);
    }
}

__device__ __forceinline__ uint4 f32_to_bf16x8(const float* f) {
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = (uint32_t)f2bf(f[2 * k]) | ((uint32_t)f2bf(f[2 * k + 1]) << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// 2x2x2 average pooling (dims even): y[b][z][y][x][c] = mean of the 8 children.
// Grid over the coarse (output) volume go, 8 channels per thread.
__global__ void k_pool_fwd(const uint16_t* x, Geo go, int C, uint16_t* y) {
    VoxG o;
    if (!vox_of(go, C / 8, o)) return;
    // children d = 4 dz + 2 dy + dx, summed as ((c0 + c1) + (c2 + c3)) +
    // ((c4 + c5) + (c6 + c7)), the order of the pool fused into the
    // row-reuse conv
    float f[8][8];
#pragma unroll
    for (int d = 0; d < 8; ++d)
        bf16x8_to_f32(*reinterpret_cast<const uint4*>(x + child(go, o, d) * C + o.grp * 8), f[d]);
    float s[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        s[k] = (((f[0][k] + f[1][k]) + (f[2][k] + f[3][k])) +
                ((f[4][k] + f[5][k]) + (f[6][k] + f[7][k]))) * 0.125f;
    *reinterpret_cast<uint4*>(y + o.v * C + o.grp * 8) = f32_to_bf16x8(s);
}

// The LeakyReLU input gradient of 4 channels, as k_lrelu_bwd computes it:
// bf16(y > 0 ? r : alpha r), stored at dz + i (8 bytes).
__device__ __forceinline__ void lrelu_dz4(float4 r, const uint16_t* y, float alpha, uint16_t* dz,
                                          long long i) {
    const uint2 yy = *reinterpret_cast<const uint2*>(y + i);
    const float y0 = __uint_as_float(yy.x << 16), y1 = __uint_as_float(yy.x & 0xFFFF0000u),
                y2 = __uint_as_float(yy.y << 16), y3 = __uint_as_float(yy.y & 0xFFFF0000u);
    uint2 o;
    o.x = (uint32_t)f2bf(y0 > 0.0f ? r.x : alpha * r.x) |
          ((uint32_t)f2bf(y1 > 0.0f ? r.y : alpha * r.y) << 16);
    o.y = (uint32_t)f2bf(y2 > 0.0f ? r.z : alpha * r.z) |
          ((uint32_t)f2bf(y3 > 0.0f ? r.w : alpha * r.w) << 16);
    *reinterpret_cast<uint2*>(dz + i) = o;
}

// Pooling backward: dx (FP32, fine grid gi, Cx channels per voxel, the first
// C used) += dy(parent) / 8, 4 channels per thread; with dz non-null the sum
// goes instead, through the LeakyReLU derivative of y (the fine level's
// activation), to dz (bf16).
__global__ void k_pool_bwd(const float* dy, Geo gi, int C, int Cx, float* dx, const uint16_t* y,
                           float alpha, uint16_t* dz) {
    VoxG f;
    if (!vox_of(gi, C / 4, f)) return;
    const float4 p = *reinterpret_cast<const float4*>(dy + parent(gi, f) * C + f.grp * 4);
    const long long i = f.v * C + f.grp * 4;
    float4* q = reinterpret_cast<float4*>(dx + f.v * Cx + f.grp * 4);
    float4 r = *q;
    r.x += 0.125f * p.x;
    r.y += 0.125f * p.y;
    r.z += 0.125f * p.z;
    r.w += 0.125f * p.w;
    if (dz) lrelu_dz4(r, y, alpha, dz, i);
    else *q = r;
}

// Nearest x2 upsampling of a coarse tensor into channels [c0, c0+C) of a fine
// tensor with Cf channels (the up half of a concatenation); grid over the
// fine volume gf, 8 channels per thread.
__global__ void k_up_fwd(const uint16_t* x, Geo gf, int C, int Cf, int c0, uint16_t* y) {
    VoxG f;
    if (!vox_of(gf, C / 8, f)) return;
    *reinterpret_cast<uint4*>(y + f.v * Cf + c0 + f.grp * 8) =
        *reinterpret_cast<const uint4*>(x + parent(gf, f) * C + f.grp * 8);
}

// Upsampling backward: dx(coarse) = sum over the 8 children of dy[.][c0 + c];
// grid over the coarse volume gc, 4 channels per thread; with dz non-null
// the sum goes instead, through the LeakyReLU derivative of y (the coarse
// level's activation), to dz (bf16).
__global__ void k_up_bwd(const float* dy, Geo gc, int C, int Cf, int c0, float* dx,
                         const uint16_t* y, float alpha, uint16_t* dz) {
    VoxG o;
    if (!vox_of(gc, C / 4, o)) return;
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int d = 0; d < 8; ++d) {
        const float4 p = *reinterpret_cast<const float4*>(dy + child(gc, o, d) * Cf + c0 + o.grp * 4);
        s.x += p.x;
        s.y += p.y;
        s.z += p.z;
        s.w += p.w;
    }
    if (dz) lrelu_dz4(s, y, alpha, dz, o.v * C + o.grp * 4);
    else *reinterpret_cast<float4*>(dx + o.v * C + o.grp * 4) = s;
}

// Copy channels [0, C) of x into channels [c0, c0+C) of y (Cf channels): the
// skip half of a concatenation (8 bf16 per thread).
__global__ void k_copy_channels(const uint16_t* x, Geo g, int C, int Cf, int c0, uint16_t* y) {
    VoxG o;
    if (!vox_of(g, C / 8, o)) return;
    *reinterpret_cast<uint4*>(y + o.v * Cf + c0 + o.grp * 8) =
        *reinterpret_cast<const uint4*>(x + o.v * C + o.grp * 8);
}

// Network input from normalised maps: x[v] = {dose, rho, 0, ...} (Cx channels).
// One voxel's input channels (Cx, a multiple of 8): dose, density, zeros,
// in 16-byte stores.
__device__ __forceinline__ void store_input_row(uint16_t* row, int Cx, float d, float r) {
    uint4* q = reinterpret_cast<uint4*>(row);
    q[0] = make_uint4((uint32_t)f2bf(d) | ((uint32_t)f2bf(r) << 16), 0u, 0u, 0u);
    for (int c = 1; c < Cx / 8; ++c) q[c] = make_uint4(0u, 0u, 0u, 0u);
}

// The network input: the Cx-channel rows x (when non-null) and the two used
// channels as one bf16 pair per voxel, x2 (when non-null).
__device__ __forceinline__ void store_input(uint16_t* x, uint32_t* x2, long long v, int Cx, float d,
                                            float r) {
    if (x) store_input_row(x + v * Cx, Cx, d, r);
    if (x2) x2[v] = (uint32_t)f2bf(d) | ((uint32_t)f2bf(r) << 16);
}

__global__ void k_assemble_f32(const float* dose, const float* rho, long long nv, int Cx,
                               uint16_t* x, uint32_t* x2, float* resid) {
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < nv;
         v += (long long)gridDim.x * blockDim.x) {
        const float d = dose[v];
        resid[v] = d;
        store_input(x, x2, v, Cx, d, rho ? rho[v] : 0.0f);
    }
}

// Network input from a dose grid [nz][ny][nx] scaled by 1 / *maxp, zero
// padded into [D][H][W] (batch 1).
__global__ void k_assemble_grid(const double* dose, const float* rho, int nx, int ny, int nz,
                                int W, int H, int D, const double* maxp, int Cx, uint16_t* x,
                                uint32_t* x2, float* resid) {
    const long long nv = (long long)W * H * D;
    const double m = *maxp;
    const double inv = m > 0.0 ? 1.0 / m : 0.0;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < nv;
         v += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(v % W), j = (int)((v / W) % H), k = (int)(v / ((long long)W * H));
        float d = 0.0f, r = 0.0f;
        if (i < nx && j < ny && k < nz) {
            const long long u = ((long long)k * ny + j) * nx + i;
            d = (float)(dose[u] * inv);
            r = rho ? rho[u] : 0.0f;
        }
        resid[v] = d;
        store_input(x, x2, v, Cx, d, r);
    }
}

// out[nz][ny][nx] = max(0, net cropped) * (*maxp)
__global__ void k_finish_grid(const float* net, int nx, int ny, int nz, int W, int H,
                              const double* maxp, double* out) {
    // thread: voxel (i, j = blockIdx.y, k = blockIdx.z) of the dose grid
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    if (i >= nx) return;
    const float y = net[((long long)k * H + j) * W + i];
    out[((long long)k * ny + j) * nx + i] = y > 0.0f ? (double)y * *maxp : 0.0;
}

// Training pair: low / m, high / m with m = *maxp (the low map's maximum),
// and the loss weight: relative error with a floor eps above the threshold
// thr, 1 / (h + eps)^2, tapering linearly to zero below it, (h / thr) /
// (thr + eps)^2, so that voxels the gamma test ignores (and their stray
// single-history deposits) do not drive the fit.
__global__ void k_prepare_pair(const double* low, const double* high, long long n,
                               const double* maxp, float eps, float thr, float* lo, float* hi,
                               float* wt) {
    const double m = *maxp;
    const double inv = m > 0.0 ? 1.0 / m : 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        lo[i] = (float)(low[i] * inv);
        if (high) {
            const float h = (float)(high[i] * inv);
            hi[i] = h;
            if (wt) {
                const float hp = fmaxf(h, 0.0f);
                const float d = hp >= thr ? hp + eps : thr + eps;
                const float r = 1.0f / (d * d);
                wt[i] = hp >= thr ? r : (hp / thr) * r;
            }
        }
    }
}

// Maximum of |a| as the bit pattern of a non-negative double (out zeroed first).
// max |a| as the bit pattern of a non-negative double (ordered like the
// value): a wave reduction, then the workgroup's 4 waves through LDS, then
// one atomic per workgroup (same-address atomics serialise in L2).
__global__ void __launch_bounds__(256) k_max_abs(const double* a, long long n,
                                                 unsigned long long* out) {
    __shared__ unsigned long long red[4];
    double m = 0.0;
    // 16-byte loads from the first 16-byte boundary; the elements before it
    // and after the last full pair are read singly
    const long long head = (reinterpret_cast<uintptr_t>(a) & 8) && n > 0 ? 1 : 0;
    const long long n2 = (n - head) / 2, stride = (long long)gridDim.x * blockDim.x;
    const double2* a2 = reinterpret_cast<const double2*>(a + head);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2; i += stride) {
        const double2 v = a2[i];
        m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (head) m = fmax(m, fabs(a[0]));
        if (head + 2 * n2 < n) m = fmax(m, fabs(a[n - 1]));
    }
    unsigned long long b = (unsigned long long)__double_as_longlong(m);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long c = __shfl_xor(b, o);
        b = c > b ? c : b;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = red[0];
        for (int k = 1; k < 4; ++k) t = red[k] > t ? red[k] : t;
        atomicMax(out, t);
    }
}

// Head: out[v] = resid[v] + b + sum_c w[c] x[v][c] (1x1x1 conv to one channel).
template <int C>
__global__ void k_head_fwd(const uint16_t* x, const float* w, const float* b, const float* resid,
                           long long nv, float* out) {
    float wr[C];
#pragma unroll
    for (int c = 0; c < C; ++c) wr[c] = w[c];
    const float bb = b[0];
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < nv;
         v += (long long)gridDim.x * blockDim.x) {
        float s = bb + resid[v];
        const uint4* xv = reinterpret_cast<const uint4*>(x + v * C);
#pragma unroll
        for (int g8 = 0; g8 < C / 8; ++g8) {
            const uint4 u = xv[g8];
            const uint32_t h[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s += wr[g8 * 8 + 2 * k] * __uint_as_float(h[k] << 16);
                s += wr[g8 * 8 + 2 * k + 1] * __uint_as_float(h[k] & 0xFFFF0000u);
            }
        }
        out[v] = s;
    }
}

// Head backward: dx[v][c] = dout[v] w[c]; per-block partial sums of dw (C) and db.
template <int C>
__global__ void __launch_bounds__(256) k_head_bwd(const float* dout, const uint16_t* x,
                                                  const float* w, long long nv, float* dx,
                                                  float* part, float alpha, uint16_t* dz) {
    // dz non-null: the gradient continues through the LeakyReLU whose output
    // x is: dz = bf16(x > 0 ? dx : alpha dx) in place of dx (lrelu_bwd's values)
    float s[C + 1];
    float wr[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        s[c] = 0.0f;
        wr[c] = w[c];
    }
    s[C] = 0.0f;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < nv;
         v += (long long)gridDim.x * blockDim.x) {
        const float d = dout[v];
        float xv[C];
#pragma unroll
        for (int g8 = 0; g8 < C / 8; ++g8)
            bf16x8_to_f32(*reinterpret_cast<const uint4*>(x + v * C + g8 * 8), xv + g8 * 8);
        if (dz) {
#pragma unroll
            for (int g8 = 0; g8 < C / 8; ++g8) {
                float t[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const float gy = d * wr[g8 * 8 + k];
                    t[k] = xv[g8 * 8 + k] > 0.0f ? gy : alpha * gy;
                }
                *reinterpret_cast<uint4*>(dz + v * C + g8 * 8) = f32_to_bf16x8(t);
            }
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) dx[v * C + c] = d * wr[c];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) s[c] += d * xv[c];
        s[C] += d;
    }
    __shared__ float red[256];
#pragma unroll
    for (int c = 0; c <= C; ++c) {
        red[threadIdx.x] = s[c];
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * (C + 1) + c] = red[0];
        __syncthreads();
    }
}

// out[c] = sum_r part[r * ncol + c] (fixed order: deterministic)

__global__ void k_fill_u32(uint32_t* p, long long n, uint32_t v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Weighted squared error: loss partials and dout = 2 m (out - tgt) / n.
__global__ void __launch_bounds__(256) k_mse(const float* out, const float* tgt, const float* wgt,
                                             long long n, float* dout, float* part) {
    float s = 0.0f;
    const float inv = 1.0f / (float)n;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const float m = wgt ? wgt[i] : 1.0f;
        const float d = out[i] - tgt[i];
        s += m * d * d;
        if (dout) dout[i] = 2.0f * m * d * inv;
    }
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] * inv;
}

// Adam (Kingma and Ba) on FP32 master weights; refreshes the bf16 copy.
__global__ void k_adam(float* p, const float* g, float* m, float* v, long long n, float lr,
                       float b1, float b2, float eps, float bc1, float bc2, uint16_t* p16) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
        p[i] = pi;
        if (p16) p16[i] = f2bf(pi);
    }
}

__global__ void k_f32_to_bf16(const float* a, long long n, uint16_t* b) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        b[i] = f2bf(a[i]);
}

inline int blocks_for(long long n, int bs = 256, int cap = 16384) {
    long long g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// The persistent row-reuse convolution: as many workgroups as the device
// holds at once (the occupancy the compiler's register and LDS use allows),
// at most one per brick.
template <int CI, int CS, int OUT>
hipError_t launch_rows_as(const uint16_t* x, const uint16_t* xl, const uint16_t* w,
                          const float* bias, Geo g, float alpha, int act, uint16_t* y16,
                          float* y32, int accumulate, hipStream_t s, HeadArgs head = {},
                          int groups = 1) {
    constexpr bool F32 = OUT == kOutF32;
    constexpr size_t lds = ((size_t)kRVox * brick_row(CI) + 256 * 8) * sizeof(uint16_t);
    static const int cap = [] {
        if (lds > 64 * 1024 &&
            hipFuncSetAttribute((const void*)k_conv_rows<CI, CS, OUT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024) != hipSuccess)
            return 0;
        int dev = 0, cu = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_conv_rows<CI, CS, OUT>, 256,
                                                         lds) != hipSuccess)
            return 0;
        return per * cu;
    }();
    if (cap <= 0) return hipErrorInvalidConfiguration;
    const long long nbk = (long long)((g.W + kRX - 1) / kRX) * ((g.H + kRY - 1) / kRY) *
                          ((g.D + kRZ - 1) / kRZ) * g.B;
    if (nbk >= (1LL << 31) || g.nvox() * 16 * groups * (F32 ? 4 : 2) >= (1LL << 31))
        return hipErrorInvalidValue;
    const int grid = (int)std::min<long long>(nbk, cap);
    hipLaunchKernelGGL((k_conv_rows<CI, CS, OUT>), dim3((unsigned)grid, groups), dim3(256), lds, s,
                       x, xl, w, bias, g, alpha, act, y16, y32, accumulate, head, 16 * groups);
    return hipGetLastError();
}

template <int CI, int CS>
hipError_t launch_rows(const uint16_t* x, const uint16_t* xl, const uint16_t* w,
                       const float* bias, Geo g, float alpha, int act, uint16_t* y16, float* y32,
                       int accumulate, hipStream_t s, int groups = 1) {
    return y32 ? launch_rows_as<CI, CS, kOutF32>(x, xl, w, bias, g, alpha, act, y16, y32,
                                                  accumulate, s, {}, groups)
               : launch_rows_as<CI, CS, kOutBf16>(x, xl, w, bias, g, alpha, act, y16, y32, 0, s,
                                                   {}, groups);
}

}  // namespace

bool conv_dz_wide_supported(int Ci, int Co, const int* dims) {
    const Geo g{dims[0], dims[1], dims[2], dims[3]};
    const int nt = (Co + 15) / 16;
    const bool few = (long long)((g.W + kRX - 1) / kRX) * ((g.H + kRY - 1) / kRY) *
                         ((g.D + kRZ - 1) / kRZ) * g.B < kFewBricks;
    if (Co == 16) return false;
    // the register kernel or the channel-pass kernel takes it (as conv_fwd routes)
    if (g.nvox() * std::max(Ci, Co) * 2 < (1LL << 31) && (Ci == 16 || Ci == 32) &&
        (nt == 2 || nt == 6 || (nt == 4 && few)))
        return true;
    return Ci % 32 == 0 && Ci >= 64 && (nt == 2 || nt == 4 || (nt % 2 == 0 && few));
}

hipError_t conv_fwd(const uint16_t* x, const uint16_t* w, const float* bias, const int* dims,
                    int Ci, int Co, float alpha, int act, uint16_t* y16, float* y32,
                    int accumulate, hipStream_t s, const uint16_t* ym) {
    Geo g{dims[0], dims[1], dims[2], dims[3]};
    const long long nv = g.nvox();
    const int nt = (Co + 15) / 16;
    if (ym && (y32 || !y16 || bias || act || accumulate || !conv_dz_wide_supported(Ci, Co, dims)))
        return hipErrorInvalidValue;
    // the halo kernel may use more than the default 64 KB of dynamic LDS
    static const hipError_t attr = [] {
        hipError_t e = hipFuncSetAttribute((const void*)k_conv_fwd_halo<1>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_conv_fwd_halo<2>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
        return e;
    }();
    if (attr != hipSuccess) return attr;
    if (nv * std::max(Ci, Co) * 2 < (1LL << 31)) {   // few channels, weights in registers
        const long long nbk = (long long)((g.W + kRX - 1) / kRX) * ((g.H + kRY - 1) / kRY) *
                              ((g.D + kRZ - 1) / kRZ) * g.B;
        // the brick, then two weight chunks of CH NT 1 KB fragments
#define LAUNCH_REG(CI, NT, CH)                                                             \
    hipLaunchKernelGGL((k_conv_fwd_reg<CI, NT, CH>), dim3((unsigned)nbk, nt / NT), dim3(256), \
                       ((size_t)kRVox * (CI + 8) + 2 * NT * CH * 512) * sizeof(uint16_t), s, x, w, \
                       bias, g, Co, alpha, act, y16, y32, accumulate, ym)
        // 16 outputs: the persistent row-reuse form (48 from 16 inputs: three
        // groups of 16, blockIdx.y)
        if (Co == 16 && Ci == 16)
            return launch_rows<16, 16>(x, nullptr, w, bias, g, alpha, act, y16, y32, accumulate, s);
        if (Co == 48 && Ci == 16)
            return launch_rows<16, 16>(x, nullptr, w, bias, g, alpha, act, y16, y32, accumulate, s,
                                       3);
        if (Co == 16 && Ci == 32)
            return launch_rows<32, 32>(x, nullptr, w, bias, g, alpha, act, y16, y32, accumulate, s);
        if (Co == 16 && Ci == 48)
            return launch_rows<48, 48>(x, nullptr, w, bias, g, alpha, act, y16, y32, accumulate, s);
        bool done = true;
        // 32 outputs, 96 as three groups of 32, or 64 as two when the bricks
        // are too few to fill the device
        const bool few = nbk < kFewBricks;
        if (Ci == 16 && (nt == 2 || nt == 6 || (nt == 4 && few))) LAUNCH_REG(16, 2, 4);
        else if (Ci == 32 && (nt == 2 || nt == 6 || (nt == 4 && few))) LAUNCH_REG(32, 2, 6);
        else done = false;
#undef LAUNCH_REG
        if (done) return hipGetLastError();
    }
    const bool few = (long long)((g.W + kRX - 1) / kRX) * ((g.H + kRY - 1) / kRY) *
                         ((g.D + kRZ - 1) / kRZ) * g.B < kFewBricks;
    if (Ci % 32 == 0 && Ci >= 64 && (nt == 2 || nt == 4 || (nt % 2 == 0 && few))) {
        // wide input, channel passes (on few bricks in groups of 32 outputs)
        const long long nbk = (long long)((g.W + kRX - 1) / kRX) * ((g.H + kRY - 1) / kRY) *
                              ((g.D + kRZ - 1) / kRZ) * g.B;
        if (nt == 2 || few)
            hipLaunchKernelGGL((k_conv_fwd_pass<2, 2>), dim3((unsigned)nbk, nt / 2), dim3(256),
                               pass_lds_bytes(2, 2), s, x, nullptr, w, bias, g, Ci, Ci, Co, alpha,
                               act, y16, y32, accumulate, ym);
        else
            hipLaunchKernelGGL((k_conv_fwd_pass<4, 2>), dim3((unsigned)nbk), dim3(256),
                               pass_lds_bytes(4, 2), s, x, nullptr, w, bias, g, Ci, Ci, Co, alpha,
                               act, y16, y32, accumulate, ym);
        return hipGetLastError();
    }
    if (nt <= 2 && Ci <= 48) {   // few channels: input brick with halo in LDS
        const size_t lds_h =
            ((size_t)kHVox * (Ci + 8) + (size_t)nt * 16 * kSlabRow) * sizeof(uint16_t);
        const long long nbk = (long long)((g.W + kHX - 1) / kHX) * ((g.H + kHY - 1) / kHY) *
                              ((g.D + kHZ - 1) / kHZ) * g.B;
        if (nt == 1)
            hipLaunchKernelGGL(k_conv_fwd_halo<1>, dim3((unsigned)nbk), dim3(256), lds_h, s, x, w,
                               bias, g, Ci, Co, alpha, act, y16, y32, accumulate);
        else
            hipLaunchKernelGGL(k_conv_fwd_halo<2>, dim3((unsigned)nbk), dim3(256), lds_h, s, x, w,
                               bias, g, Ci, Co, alpha, act, y16, y32, accumulate);
        return hipGetLastError();
    }
    const size_t lds = (size_t)nt * 16 * kSlabRow * sizeof(uint16_t);
#define LAUNCH(NT, MT)                                                                        \
    hipLaunchKernelGGL((k_conv_fwd_lds<NT, MT>), dim3((unsigned)((nv + 64 * MT - 1) / (64 * MT))), \
                       dim3(256), lds, s, x, w, bias, g, Ci, Co, alpha, act, y16, y32, accumulate)
    if (nt % 2 == 0 && nt > 2 && (nv + 127) / 128 < 512) {
        // few voxels (the coarsest level): split the output channels over
        // blockIdx.y so the launch still fills the device
        hipLaunchKernelGGL((k_conv_fwd_lds<2, 2>), dim3((unsigned)((nv + 127) / 128), nt / 2),
                           dim3(256), (size_t)2 * 16 * kSlabRow * sizeof(uint16_t), s, x, w, bias,
                           g, Ci, Co, alpha, act, y16, y32, accumulate);
        return hipGetLastError();
    }
    switch (nt) {
        case 1: LAUNCH(1, 4); break;
        case 2: LAUNCH(2, 4); break;
        case 3: LAUNCH(3, 4); break;
        case 4: LAUNCH(4, 4); break;
        case 6: LAUNCH(6, 2); break;
        case 8: LAUNCH(8, 2); break;
        case 12: LAUNCH(12, 2); break;
        default: return hipErrorInvalidValue;
    }
#undef LAUNCH
    return hipGetLastError();
}

bool conv_cat_fwd_supported(int Cs, int Cu, int Co, long long nvox) {
    if (nvox * (Cs + Cu) * 2 >= (1LL << 31)) return false;   // 32-bit buffer offsets
    if (Cs == 16 && Cu == 32 && Co == 16) return true;
    return Cs % 8 == 0 && Cu % 8 == 0 && (Cs + Cu) % 32 == 0 && Cs + Cu >= 64 &&
           (Co == 32 || Co == 64);
}

hipError_t conv_cat_fwd(const uint16_t* skip, const uint16_t* low, const uint16_t* w,
                        const float* bias, const int* dims, int Cs, int Cu, int Co, float alpha,
                        int act, uint16_t* y16, hipStream_t s) {
    Geo g{dims[0], dims[1], dims[2], dims[3]};
    if (!conv_cat_fwd_supported(Cs, Cu, Co, g.nvox()) || (g.D | g.H | g.W) & 1 || !y16)
        return hipErrorInvalidValue;
    const long long nbk = (long long)((g.W + kRX - 1) / kRX) * ((g.H + kRY - 1) / kRY) *
                          ((g.D + kRZ - 1) / kRZ) * g.B;
    if (Co == 32 || Co == 64) {
        if (Co == 32 || nbk < kFewBricks)   // 64 outputs on few bricks: two groups of 32
            hipLaunchKernelGGL((k_conv_fwd_pass<2, 2>), dim3((unsigned)nbk, Co / 32), dim3(256),
                               pass_lds_bytes(2, 2), s, skip, low, w, bias, g, Cs + Cu, Cs, Co,
                               alpha, act, y16, nullptr, 0, nullptr);
        else
            hipLaunchKernelGGL((k_conv_fwd_pass<4, 2>), dim3((unsigned)nbk), dim3(256),
                               pass_lds_bytes(4, 2), s, skip, low, w, bias, g, Cs + Cu, Cs, Co,
                               alpha, act, y16, nullptr, 0, nullptr);
        return hipGetLastError();
    }
    return launch_rows<48, 16>(skip, low, w, bias, g, alpha, act, y16, nullptr, 0, s);
}

hipError_t conv_fwd_split(const uint16_t* x, const uint16_t* w, const int* dims, int Ci, int Co,
                          int cs, float* ya, const uint16_t* ym, float alpha, uint16_t* dzc,
                          hipStream_t s) {
    Geo g{dims[0], dims[1], dims[2], dims[3]};
    const Geo gc{g.B, g.D >> 1, g.H >> 1, g.W >> 1};
    if (Ci != 16 || Co != 48 || cs != 16 || !ym || !dzc || ((g.D | g.H | g.W) & 1) ||
        gc.nvox() * 32 * 2 >= (1LL << 31) || dzc == x)
        return hipErrorInvalidValue;
    if (ya) {
        hipError_t e = launch_rows<16, 16>(x, nullptr, w, nullptr, g, 0.0f, 0, nullptr, ya, 0, s, 1);
        if (e != hipSuccess) return e;
    }
    HeadArgs a{};
    a.ym = ym;
    a.pool = dzc;
    return launch_rows_as<16, 16, kOutUpDz>(x, nullptr, w + 16LL * 27 * 16, nullptr, g, alpha, 0,
                                            nullptr, nullptr, 0, s, a, 2);
}

hipError_t conv_pool_fwd(const uint16_t* x, const uint16_t* w, const float* bias, const int* dims,
                         float alpha, uint16_t* y16, uint16_t* pool, hipStream_t s) {
    Geo g{dims[0], dims[1], dims[2], dims[3]};
    if (g.nvox() * 16 * 2 >= (1LL << 31) || !y16 || !pool || ((g.D | g.H | g.W) & 1))
        return hipErrorInvalidValue;
    HeadArgs a{};
    a.pool = pool;
    return launch_rows_as<16, 16, kOutPool>(x, nullptr, w, bias, g, alpha, 1, y16, nullptr, 0, s,
                                            a);
}

hipError_t conv_dz_fwd(const uint16_t* x, const uint16_t* w, const int* dims, const uint16_t* ym,
                       float alpha, uint16_t* dz, hipStream_t s, const float* par) {
    Geo g{dims[0], dims[1], dims[2], dims[3]};
    if (g.nvox() * 16 * 2 >= (1LL << 31) || !ym || !dz || dz == x ||
        (par && ((g.D | g.H | g.W) & 1)))
        return hipErrorInvalidValue;
    HeadArgs a{};
    a.ym = ym;
    a.par = par;
    return launch_rows_as<16, 16, kOutDz>(x, nullptr, w, nullptr, g, alpha, 0, dz, nullptr, 0, s, a);
}

hipError_t conv_head_fwd(const uint16_t* x, const uint16_t* w, const float* bias, const int* dims,
                         float alpha, uint16_t* y16, const float* head_w, const float* head_b,
                         const float* resid, float* out, hipStream_t s) {
    Geo g{dims[0], dims[1], dims[2], dims[3]};
    if (g.nvox() * 16 * 2 >= (1LL << 31)) return hipErrorInvalidValue;
    return launch_rows_as<16, 16, kOutHead>(x, nullptr, w, bias, g, alpha, 1, y16, nullptr, 0, s,
                                            HeadArgs{head_w, head_b, resid, out, nullptr, nullptr});
}

hipError_t conv_in_fwd(const uint32_t* x2, const uint16_t* w, int cin, const float* bias,
                       const int* dims, float alpha, uint16_t* y16, hipStream_t s) {
    Geo g{dims[0], dims[1], dims[2], dims[3]};
    if (cin < 2 || !y16 || g.nvox() * 16 * 2 >= (1LL << 31)) return hipErrorInvalidValue;
    static const int cap = [] {
        int dev = 0, cu = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_conv_in, 256, 0) != hipSuccess)
            return 0;
        return per * cu;
    }();
    if (cap <= 0) return hipErrorInvalidConfiguration;
    const long long nbk = (long long)((g.W + kRX - 1) / kRX) * ((g.H + kRY - 1) / kRY) *
                          ((g.D + kRZ - 1) / kRZ) * g.B;
    const int grid = (int)std::min<long long>(nbk, cap);
    hipLaunchKernelGGL(k_conv_in, dim3((unsigned)grid), dim3(256), 0, s, x2, w, cin, bias, g, alpha,
                       y16);
    return hipGetLastError();
}

// Every layer's flip in one launch: thread i handles element i of the
// concatenation of the layers' weights (job k covers [start[k], start[k + 1])).
__global__ void k_flip_all(FlipJobs jobs) {
    const long long n = jobs.start[jobs.n];
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        int k = 0;
        while (k + 1 < jobs.n && i >= jobs.start[k + 1]) ++k;
        const int e = (int)(i - jobs.start[k]), Ci = jobs.ci[k], Co = jobs.co[k];
        const int ci = e % Ci, t = (e / Ci) % 27, co = e / (27 * Ci);
        jobs.wt[k][((size_t)ci * 27 + (26 - t)) * Co + co] = jobs.w[k][e];
    }
}

hipError_t flip_transpose_all(const FlipJobs& jobs, hipStream_t s) {
    if (jobs.n < 1 || jobs.n > kMaxFlipJobs) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_flip_all, dim3(blocks_for(jobs.start[jobs.n])), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

hipError_t flip_transpose(const uint16_t* w, uint16_t* wt, int Ci, int Co, hipStream_t s) {
    hipLaunchKernelGGL(k_flip_transpose, dim3(blocks_for((long long)Co * 27 * Ci)), dim3(256), 0, s,
                       w, wt, Ci, Co);
    return hipGetLastError();
}

long long wgrad_chunks(const int* dims, int chunk) {
    const long long nv = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    return (nv + chunk - 1) / chunk;
}

// Chunk length (a multiple of the 64-voxel slice) giving about 1024
// workgroups in all, within max_part_floats of partial sums.
int wgrad_chunk_for(const int* dims, int Ci, int Co, long long max_part_floats) {
    const long long nv = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    const int tg = wgrad_taps_per_group(Ci, Co);
    const long long groups = (27 + tg - 1) / tg;
    long long target = (1024 + groups - 1) / groups;
    const long long cap = max_part_floats / (27LL * Ci * Co + Co);
    if (target > cap) target = cap;
    if (target < 1) target = 1;
    long long chunk = (nv + target - 1) / target;
    chunk = (chunk + kWgSlice - 1) / kWgSlice * kWgSlice;
    if (chunk < kWgSlice) chunk = kWgSlice;
    return (int)chunk;
}

long long wgrad_part_floats(const int* dims, int Ci, int Co, int chunk) {
    return wgrad_chunks(dims, chunk) * (27LL * Ci * Co + Co);
}

namespace {
bool wgrad_by_bricks(const Geo& g, int Ci, int Co) {
    return (Co == 16 || Co == 32 || Co == 64 || Co == 128) &&
           g.nvox() * std::max(Ci, Co) * 2 < (1LL << 31);
}

// x: Cs channels per voxel; xl (the half-size level, Ci - Cs channels) when Cs < Ci
hipError_t wgrad_impl(const uint16_t* dz, const uint16_t* x, const uint16_t* xl, const int* dims,
                      int Ci, int Cs, int Co, int chunk, float* part, float* dw, float* db,
                      hipStream_t s) {
    Geo g{dims[0], dims[1], dims[2], dims[3]};
    long long nchunk = wgrad_chunks(dims, chunk);
    if (wgrad_by_bricks(g, Ci, Co)) {
        // by bricks, within the same partial-sum buffer (32-bit buffer offsets);
        // 64 or 128 outputs as groups of 32, each with its own partials
        static const hipError_t attr = [] {
            hipError_t e = hipFuncSetAttribute((const void*)k_wgrad_brick<1>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
            if (e == hipSuccess)
                e = hipFuncSetAttribute((const void*)k_wgrad_brick<2>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
            return e;
        }();
        if (attr != hipSuccess) return attr;
        const long long nbk = (long long)((g.W + kRX - 1) / kRX) * ((g.H + kRY - 1) / kRY) *
                              ((g.D + kRZ - 1) / kRZ) * g.B;
        if (nbk > (1LL << 30)) return hipErrorInvalidValue;
        // about 512 workgroups per launch (two per CU, one round): fewer
        // split-K rows for the column sums, more bricks per workgroup to
        // pipeline
        const long long want =
            std::max(1LL, std::min({nchunk, nbk, 512LL / std::max(1, Ci / 16)}));
        const int bpc = (int)((nbk + want - 1) / want);
        const long long used = (nbk + bpc - 1) / bpc;   // <= nchunk
        float* part_b = part + used * 27LL * Co * Ci;
        const int cg = Co == 16 ? 16 : 32;   // outputs per group
        for (int co0 = 0; co0 < Co; co0 += cg) {
            float* pw = part + used * 27LL * co0 * Ci;
            float* pb = part_b + used * co0;
            const size_t lds = (size_t)wgrad_brick_lds_bytes(cg);
            if (cg == 16)
                hipLaunchKernelGGL(k_wgrad_brick<1>, dim3((unsigned)used, Ci / 16), dim3(256), lds,
                                   s, dz + co0, x, xl, g, Ci, Cs, bpc, (int)nbk, pw, pb, Co);
            else
                hipLaunchKernelGGL(k_wgrad_brick<2>, dim3((unsigned)used, Ci / 16), dim3(256), lds,
                                   s, dz + co0, x, xl, g, Ci, Cs, bpc, (int)nbk, pw, pb, Co);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        const int n = 27 * Co * Ci, nbw = (n + 63) / 64;
        hipLaunchKernelGGL(k_colsum_wb, dim3(nbw + (db ? (Co + 63) / 64 : 0)), dim3(1024), 0, s,
                           part, part_b, (int)used, n, nbw, Co, dw, db, (Ci << 16) | cg);
        return hipGetLastError();
    }
    if (Cs != Ci) return hipErrorInvalidValue;   // a concatenation is read in place by bricks only
    const int tg = wgrad_taps_per_group(Ci, Co);
    const int groups = (27 + tg - 1) / tg;
    if (tg * (Co / 16) * (Ci / 16) > kWgWaves * kWgMaxTiles && tg > 1) return hipErrorInvalidValue;
    if ((Co / 16) * (Ci / 16) > kWgWaves * kWgMaxTiles) return hipErrorInvalidValue;
    const size_t lds = (size_t)(Co + tg * Ci) * kWgRow * sizeof(uint16_t);
    float* part_b = part + nchunk * 27LL * Co * Ci;
    hipLaunchKernelGGL(k_wgrad_partial, dim3((unsigned)nchunk, groups), dim3(64 * kWgWaves), lds, s,
                       dz, x, g, Ci, Co, chunk, tg, part, part_b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n = 27 * Co * Ci, nbw = (n + 63) / 64;
    hipLaunchKernelGGL(k_colsum_wb, dim3(nbw + (db ? (Co + 63) / 64 : 0)), dim3(1024), 0, s, part,
                       part_b, (int)nchunk, n, nbw, Co, dw, db, (Ci << 16) | Co);
    return hipGetLastError();
}
}  // namespace

hipError_t wgrad(const uint16_t* dz, const uint16_t* x, const int* dims, int Ci, int Co, int chunk,
                 float* part, float* dw, float* db, hipStream_t s) {
    return wgrad_impl(dz, x, nullptr, dims, Ci, Ci, Co, chunk, part, dw, db, s);
}

bool wgrad_cat_supported(int Cs, int Cu, int Co, const int* dims) {
    const Geo g{dims[0], dims[1], dims[2], dims[3]};
    return Cs > 0 && Cu > 0 && Cs % 16 == 0 && Cu % 16 == 0 && ((g.D | g.H | g.W) & 1) == 0 &&
           wgrad_by_bricks(g, Cs + Cu, Co);
}

hipError_t wgrad_cat(const uint16_t* dz, const uint16_t* skip, const uint16_t* low,
                     const int* dims, int Cs, int Cu, int Co, int chunk, float* part, float* dw,
                     float* db, hipStream_t s) {
    if (!wgrad_cat_supported(Cs, Cu, Co, dims)) return hipErrorInvalidValue;
    return wgrad_impl(dz, skip, low, dims, Cs + Cu, Cs, Co, chunk, part, dw, db, s);
}

hipError_t lrelu_bwd(const float* dy, const uint16_t* y, float alpha, long long n, uint16_t* dz,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_lrelu_bwd, dim3(blocks_for(n)), dim3(256), 0, s, dy, y, alpha, n, dz);
    return hipGetLastError();
}

hipError_t pool_fwd(const uint16_t* x, const int* dims_out, int C, uint16_t* y, hipStream_t s) {
    Geo g{dims_out[0], dims_out[1], dims_out[2], dims_out[3]};
    if (C % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pool_fwd, vox_grid(g, C / 8), dim3(256), 0, s, x, g, C, y);
    return hipGetLastError();
}

hipError_t pool_bwd(const float* dy, const int* dims_in, int C, float* dx, hipStream_t s,
                    const uint16_t* y, float alpha, uint16_t* dz, int cx) {
    Geo g{dims_in[0], dims_in[1], dims_in[2], dims_in[3]};
    if (cx == 0) cx = C;
    if (C % 4 || cx % 4 || cx < C || (dz && !y)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pool_bwd, vox_grid(g, C / 4), dim3(256), 0, s, dy, g, C, cx, dx, y,
                       alpha, dz);
    return hipGetLastError();
}

hipError_t up_fwd(const uint16_t* x, const int* dims_fine, int C, int Cf, int c0, uint16_t* y,
                  hipStream_t s) {
    Geo g{dims_fine[0], dims_fine[1], dims_fine[2], dims_fine[3]};
    if (C % 8 || Cf % 8 || c0 % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_up_fwd, vox_grid(g, C / 8), dim3(256), 0, s, x, g, C, Cf, c0, y);
    return hipGetLastError();
}

hipError_t up_bwd(const float* dy, const int* dims_coarse, int C, int Cf, int c0, float* dx,
                  hipStream_t s, const uint16_t* y, float alpha, uint16_t* dz) {
    Geo g{dims_coarse[0], dims_coarse[1], dims_coarse[2], dims_coarse[3]};
    if (C % 4 || Cf % 4 || c0 % 4 || (dz && !y)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_up_bwd, vox_grid(g, C / 4), dim3(256), 0, s, dy, g, C, Cf, c0, dx, y,
                       alpha, dz);
    return hipGetLastError();
}

hipError_t copy_channels(const uint16_t* x, const int* dims, int C, int Cf, int c0, uint16_t* y,
                         hipStream_t s) {
    Geo g{dims[0], dims[1], dims[2], dims[3]};
    if (C % 8 || Cf % 8 || c0 % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy_channels, vox_grid(g, C / 8), dim3(256), 0, s, x, g, C, Cf, c0, y);
    return hipGetLastError();
}

hipError_t assemble_f32(const float* dose, const float* rho, long long nv, int Cx, uint16_t* x,
                        uint32_t* x2, float* resid, hipStream_t s) {
    if (Cx < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_assemble_f32, dim3(blocks_for(nv)), dim3(256), 0, s, dose, rho, nv, Cx, x,
                       x2, resid);
    return hipGetLastError();
}

hipError_t assemble_grid(const double* dose, const float* rho, const int* src, const int* dst,
                         const double* maxp, int Cx, uint16_t* x, uint32_t* x2, float* resid,
                         hipStream_t s) {
    if (Cx < 2) return hipErrorInvalidValue;
    const long long nv = (long long)dst[0] * dst[1] * dst[2];
    hipLaunchKernelGGL(k_assemble_grid, dim3(blocks_for(nv)), dim3(256), 0, s, dose, rho, src[2],
                       src[1], src[0], dst[2], dst[1], dst[0], maxp, Cx, x, x2, resid);
    return hipGetLastError();
}

hipError_t finish_grid(const float* net, const int* src, const int* dst, const double* maxp,
                       double* out, hipStream_t s) {
    if (src[0] > 65535 || src[1] > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_finish_grid, dim3((unsigned)((src[2] + 255) / 256), src[1], src[0]),
                       dim3(256), 0, s, net, src[2], src[1], src[0], dst[2], dst[1], maxp, out);
    return hipGetLastError();
}

hipError_t prepare_pair(const double* low, const double* high, long long n, const double* maxp,
                        float eps, float thr, float* lo, float* hi, float* wt, hipStream_t s) {
    hipLaunchKernelGGL(k_prepare_pair, dim3(blocks_for(n)), dim3(256), 0, s, low, high, n, maxp, eps,
                       thr, lo, hi, wt);
    return hipGetLastError();
}

hipError_t max_abs(const double* a, long long n, unsigned long long* out_bits, hipStream_t s) {
    hipLaunchKernelGGL(k_max_abs, dim3(blocks_for(n, 256, 1024)), dim3(256), 0, s, a, n, out_bits);
    return hipGetLastError();
}

hipError_t head_fwd(const uint16_t* x, const float* w, const float* b, const float* resid,
                    long long nv, int C, float* out, hipStream_t s) {
    if (C == 16)
        hipLaunchKernelGGL(k_head_fwd<16>, dim3(blocks_for(nv)), dim3(256), 0, s, x, w, b, resid, nv, out);
    else if (C == 32)
        hipLaunchKernelGGL(k_head_fwd<32>, dim3(blocks_for(nv)), dim3(256), 0, s, x, w, b, resid, nv, out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

int head_bwd_blocks(long long nv) { return blocks_for(nv, 256, 1024); }

hipError_t head_bwd(const float* dout, const uint16_t* x, const float* w, long long nv, int C,
                    float* dx, float* part, hipStream_t s, float alpha, uint16_t* dz) {
    const int g = head_bwd_blocks(nv);
    if (C == 16)
        hipLaunchKernelGGL(k_head_bwd<16>, dim3(g), dim3(256), 0, s, dout, x, w, nv, dx, part,
                           alpha, dz);
    else if (C == 32)
        hipLaunchKernelGGL(k_head_bwd<32>, dim3(g), dim3(256), 0, s, dout, x, w, nv, dx, part,
                           alpha, dz);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t sum_rows(const float* part, int nrow, int ncol, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3((ncol + 63) / 64), dim3(1024), 0, s, part, nrow, ncol, out, 0);
    return hipGetLastError();
}

hipError_t fill_u32(uint32_t* p, long long n, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

int mse_blocks(long long n) { return blocks_for(n, 256, 1024); }

hipError_t mse(const float* out, const float* tgt, const float* wgt, long long n, float* dout,
               float* part, hipStream_t s) {
    hipLaunchKernelGGL(k_mse, dim3(mse_blocks(n)), dim3(256), 0, s, out, tgt, wgt, n, dout, part);
    return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1,
                float b2, float eps, int step, uint16_t* p16, hipStream_t s) {
    const float bc1 = 1.0f - powf(b1, (float)step), bc2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                       bc1, bc2, p16);
    return hipGetLastError();
}

hipError_t f32_to_bf16(const float* a, long long n, uint16_t* b, hipStream_t s) {
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(blocks_for(n)), dim3(256), 0, s, a, n, b);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace sde

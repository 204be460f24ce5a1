// Microbenchmarks of the transport kernel's ingredients on gfx950: VALU
// issue (FMA, each transcendental, the two mixed, 32x32->64 products), int64
// atomics in global memory and LDS, and an HBM stream.  Each kernel runs a
// fixed, exactly known amount of work; the host entry point times it with
// HIP events on the library's stream.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "sde.h"
#include "sde_roofs.h"

namespace sde {
hipStream_t library_stream();
int report_error(int code, const char* msg);
}  // namespace sde

namespace {

// Results that the compiler must not drop are stored to `sink` (1024 words,
// passed as an argument so that the store cannot be proven dead) only when a
// value that cannot occur appears, so in practice nothing is written.

constexpr float kNever = -1.2345e-30f;

__global__ __launch_bounds__(1024) void k_mb_fma(float b, float c, int iters, float* sink) {
    float a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (float)(threadIdx.x & 7) * 1e-3f + (float)j;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = fmaf(a[j], b, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j];
    if (s == kNever) sink[threadIdx.x & 1023] = s;
}

// integer chains a = (a << 1) + m: one full-rate v_lshl_add_u32 each
__global__ __launch_bounds__(1024) void k_mb_int(uint32_t m, int iters, uint32_t* sink) {
    uint32_t a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = threadIdx.x * 2654435761u + (uint32_t)j;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = (a[j] << 1) + m;
    }
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s ^= a[j];
    if (s == 0x9E3779B9u && a[0] == 0x7F4A7C15u) sink[threadIdx.x & 1023] = s;
}

// float chains a = a * b (OP 0) or a = a + b (OP 1); integer chains
// a_j = a_j ^ a_{j+1} (OP 2, bitwise, mixing the chains)
template <int OP>
__global__ __launch_bounds__(1024) void k_mb_op(float b, int iters, float* sink) {
    float a[8];
    uint32_t u[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = 1.0f + (float)(threadIdx.x & 7) * 1e-3f + 0.125f * (float)j;
        u[j] = threadIdx.x * 2654435761u + (uint32_t)j * 40503u;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if constexpr (OP == 0) a[j] = a[j] * b;
            if constexpr (OP == 1) a[j] = a[j] + b;
            if constexpr (OP == 2) u[j] = u[j] ^ u[(j + 1) & 7];
        }
    }
    float s = 0.0f;
    uint32_t x = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        s += a[j];
        x ^= u[j];
    }
    if (s == kNever || x == 0x9E3779B9u) sink[threadIdx.x & 1023] = s;
}

template <int OP>
__device__ __forceinline__ float trans(float x) {
    if constexpr (OP == 0) return __builtin_amdgcn_exp2f(x);
    if constexpr (OP == 1) return __builtin_amdgcn_logf(x);
    if constexpr (OP == 2) return __builtin_amdgcn_rcpf(x);
    if constexpr (OP == 3) return __builtin_amdgcn_sqrtf(x);
    if constexpr (OP == 4) return __builtin_amdgcn_rsqf(x);
    return __builtin_amdgcn_sinf(x);
}

template <int OP>
__global__ __launch_bounds__(1024) void k_mb_trans(float x0, int iters, float* sink) {
    float a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = x0 + (float)(threadIdx.x & 7) * 1e-3f + 0.125f * (float)j;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = trans<OP>(a[j]);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j];
    if (s == kNever) sink[threadIdx.x & 1023] = s;
}

// four square-root chains beside 4 K FMA chains
template <int K>
__global__ __launch_bounds__(1024) void k_mb_mix(float b, float c, int iters, float* sink) {
    float t[4], f[4 * K];
#pragma unroll
    for (int j = 0; j < 4; ++j) t[j] = 2.0f + (float)j + (float)(threadIdx.x & 7);
#pragma unroll
    for (int j = 0; j < 4 * K; ++j) f[j] = (float)j * 0.5f + (float)(threadIdx.x & 3);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) t[j] = __builtin_amdgcn_sqrtf(t[j]);
#pragma unroll
        for (int j = 0; j < 4 * K; ++j) f[j] = fmaf(f[j], b, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) s += t[j];
#pragma unroll
    for (int j = 0; j < 4 * K; ++j) s += f[j];
    if (s == kNever) sink[threadIdx.x & 1023] = s;
}

// 32 x 32 -> 64 products (the Philox round's): chains a = hi32(a m + c),
// one v_mad_u64_u32 each
__global__ __launch_bounds__(1024) void k_mb_mul64(uint32_t m, uint32_t k, int iters, uint32_t* sink) {
    uint32_t a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = threadIdx.x * 2654435761u + (uint32_t)j * 40503u;
    const uint64_t c = ((uint64_t)k << 32) | k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = (uint32_t)(((uint64_t)a[j] * m + c) >> 32);
    }
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s ^= a[j];
    if (s == 0x9E3779B9u && a[0] == 0x7F4A7C15u) sink[threadIdx.x & 1023] = s;
}

__device__ __forceinline__ uint32_t xorshift(uint32_t x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

// int64 adds without return: mode 0 one address, 1 one address per wave
// (words 32 apart), 2 random words in [0, mask]
__global__ __launch_bounds__(1024) void k_mb_gatomic(unsigned long long* buf, uint64_t mask,
                                                     int mode, int iters) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t r = gid * 2654435761u + 0x6D2B79F5u;
    const uint64_t wave_word = ((uint64_t)(gid >> 6) * 32u) & mask;
    for (int i = 0; i < iters; ++i) {
        uint64_t w = 0;
        if (mode == 1) w = wave_word;
        if (mode == 2) {
            r = xorshift(r);
            w = (uint64_t)r & mask;
        }
        atomicAdd(buf + w, 1ull);
    }
}

__global__ __launch_bounds__(1024) void k_mb_latomic(int mode, int iters, uint32_t* sink) {
    __shared__ unsigned long long tile[8192];   // 64 KiB
    for (int i = threadIdx.x; i < 8192; i += blockDim.x) tile[i] = 0;
    __syncthreads();
    uint32_t r = (blockIdx.x * blockDim.x + threadIdx.x) * 2654435761u + 0x6D2B79F5u;
    for (int i = 0; i < iters; ++i) {
        uint32_t w = 0;
        if (mode == 2) {
            r = xorshift(r);
            w = r & 8191u;
        }
        atomicAdd(tile + w, 1ull);
    }
    __syncthreads();
    const unsigned long long v = tile[threadIdx.x & 8191];
    if (v == 0xFFFFFFFFFFFFFFFFull) sink[threadIdx.x & 1023] = (uint32_t)v;
}

// 16-byte accesses over n4 float4 words, grid-stride
__global__ __launch_bounds__(1024) void k_mb_read(const float4* __restrict__ p, uint64_t n4, float* sink) {
    float4 s = {0.0f, 0.0f, 0.0f, 0.0f};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {   // four loads in flight
        const float4 v0 = p[i], v1 = p[i + stride], v2 = p[i + 2 * stride], v3 = p[i + 3 * stride];
        s.x += (v0.x + v1.x) + (v2.x + v3.x);
        s.y += (v0.y + v1.y) + (v2.y + v3.y);
        s.z += (v0.z + v1.z) + (v2.z + v3.z);
        s.w += (v0.w + v1.w) + (v2.w + v3.w);
    }
    for (; i < n4; i += stride) {
        const float4 v = p[i];
        s.x += v.x;
        s.y += v.y;
        s.z += v.z;
        s.w += v.w;
    }
    const float t = s.x + s.y + s.z + s.w;
    if (t == kNever) sink[threadIdx.x & 1023] = t;
}

__global__ __launch_bounds__(1024) void k_mb_write(float4* __restrict__ p, uint64_t n4) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const float4 v = {1.0f, 2.0f, 3.0f, 4.0f};
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) p[i] = v;
}

__global__ __launch_bounds__(1024) void k_mb_copy(const float4* __restrict__ src,
                                                  float4* __restrict__ dst, uint64_t n4) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        dst[i] = src[i];
}

int bad(const std::string& m) { return sde::report_error(SDE_E_INVALID, m.c_str()); }

}  // namespace

extern "C" int sde_microbench(int kind, int variant, void* buf, size_t buf_bytes, int grid,
                              int block, int64_t iters, int reps, double* units_out,
                              double* ms_out) {
    if (!units_out || !ms_out) return bad("null output");
    if (block < 64 || block > 1024 || block % 64) return bad("block must be a multiple of 64 in 64..1024");
    if (grid < 1 || grid > (1 << 20)) return bad("grid must be in 1..2^20");
    if (reps < 1 || reps > 100) return bad("reps must be in 1..100");
    if (kind != SDE_MB_HBM && (iters < 1 || iters > (1 << 24)))
        return bad("iters must be in 1..2^24");
    const double lanes = (double)grid * block;
    const int it = (int)iters;
    double units = 0.0;
    uint64_t n4 = 0, mask = 0;
    switch (kind) {
        case SDE_MB_FMA:
            if (variant < 0 || variant > 4) return bad("unknown variant");
            units = lanes * it * 8.0;
            break;
        case SDE_MB_TRANS:
            if (variant < 0 || variant > 5) return bad("unknown variant");
            units = lanes * it * 8.0;
            break;
        case SDE_MB_MIX:
            if (variant != 1 && variant != 2 && variant != 4 && variant != 8) return bad("unknown variant");
            units = lanes * it * (4.0 + 4.0 * variant);
            break;
        case SDE_MB_MUL64:
            if (variant != 0) return bad("unknown variant");
            units = lanes * it * 8.0;
            break;
        case SDE_MB_GATOMIC: {
            if (variant < 0 || variant > 2) return bad("unknown variant");
            if (!buf || buf_bytes < 8 || ((uintptr_t)buf & 15)) return bad("a 16-byte aligned buffer of >= 8 bytes is needed");
            uint64_t words = buf_bytes / 8, p2 = 1;
            while (p2 * 2 <= words) p2 *= 2;
            mask = p2 - 1;
            units = lanes * it;
            break;
        }
        case SDE_MB_LATOMIC:
            if (variant != 0 && variant != 2) return bad("unknown variant");
            units = lanes * it;
            break;
        case SDE_MB_HBM:
            if (variant < 0 || variant > 2) return bad("unknown variant");
            if (!buf || buf_bytes < (1u << 20) || buf_bytes % 32 || ((uintptr_t)buf & 15))
                return bad("HBM stream needs a 16-byte aligned buffer of >= 1 MiB, a multiple of 32 bytes");
            n4 = variant == 2 ? buf_bytes / 32 : buf_bytes / 16;
            units = variant == 2 ? 2.0 * (double)n4 * 16.0 : (double)n4 * 16.0;
            break;
        default:
            return bad("unknown microbenchmark kind");
    }
    // the sink: 4 KiB, allocated on first use per device and kept
    static void* sinks[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return sde::report_error(SDE_E_HIP, "microbenchmark: no current device");
    if (!sinks[dev] && hipMalloc(&sinks[dev], 4096) != hipSuccess) {
        sinks[dev] = nullptr;
        return sde::report_error(SDE_E_NOMEM, "microbenchmark: sink allocation failed");
    }
    float* sf = (float*)sinks[dev];
    uint32_t* su = (uint32_t*)sinks[dev];
    hipStream_t s = sde::library_stream();
    auto launch = [&]() {
        const dim3 g(grid), b(block);
        switch (kind) {
            case SDE_MB_FMA:
                if (variant == 0) k_mb_fma<<<g, b, 0, s>>>(0.999f, 0.001f, it, sf);
                else if (variant == 1) k_mb_int<<<g, b, 0, s>>>(0x6D2B79F5u, it, su);
                else if (variant == 2) k_mb_op<0><<<g, b, 0, s>>>(0.99999f, it, sf);
                else if (variant == 3) k_mb_op<1><<<g, b, 0, s>>>(1e-7f, it, sf);
                else k_mb_op<2><<<g, b, 0, s>>>(0.0f, it, sf);
                break;
            case SDE_MB_TRANS:
                switch (variant) {
                    case 0: k_mb_trans<0><<<g, b, 0, s>>>(-1.0f, it, sf); break;
                    case 1: k_mb_trans<1><<<g, b, 0, s>>>(1.5f, it, sf); break;
                    case 2: k_mb_trans<2><<<g, b, 0, s>>>(1.5f, it, sf); break;
                    case 3: k_mb_trans<3><<<g, b, 0, s>>>(1.5f, it, sf); break;
                    case 4: k_mb_trans<4><<<g, b, 0, s>>>(1.5f, it, sf); break;
                    default: k_mb_trans<5><<<g, b, 0, s>>>(0.3f, it, sf); break;
                }
                break;
            case SDE_MB_MIX:
                switch (variant) {
                    case 1: k_mb_mix<1><<<g, b, 0, s>>>(0.999f, 0.001f, it, sf); break;
                    case 2: k_mb_mix<2><<<g, b, 0, s>>>(0.999f, 0.001f, it, sf); break;
                    case 4: k_mb_mix<4><<<g, b, 0, s>>>(0.999f, 0.001f, it, sf); break;
                    default: k_mb_mix<8><<<g, b, 0, s>>>(0.999f, 0.001f, it, sf); break;
                }
                break;
            case SDE_MB_MUL64: k_mb_mul64<<<g, b, 0, s>>>(0xD2511F53u, 0x9E3779B9u, it, su); break;
            case SDE_MB_GATOMIC:
                k_mb_gatomic<<<g, b, 0, s>>>((unsigned long long*)buf, mask, variant, it);
                break;
            case SDE_MB_LATOMIC: k_mb_latomic<<<g, b, 0, s>>>(variant, it, su); break;
            default:
                if (variant == 0) k_mb_read<<<g, b, 0, s>>>((const float4*)buf, n4, sf);
                else if (variant == 1) k_mb_write<<<g, b, 0, s>>>((float4*)buf, n4);
                else k_mb_copy<<<g, b, 0, s>>>((const float4*)buf, (float4*)buf + n4, n4);
                break;
        }
        return hipGetLastError();
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch();                       // untimed
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess)
        return sde::report_error(SDE_E_HIP, (std::string("microbenchmark: ") + hipGetErrorString(e)).c_str());
    *units_out = units;
    *ms_out = (double)ms / reps;
    return SDE_OK;
}

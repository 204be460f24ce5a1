// HIP kernels of the gamma index (section 2.2.3) and the array maximum it
// normalises by, for gfx950.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sde_internal.hpp"

namespace sde {
namespace {

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Gamma index, one thread per reference voxel.  off[k] = (ox / dx, oy / dy,
// oz / dz, |o|^2 / dta^2) for the lattice offsets o of spacing dta/interp
// within dta, sorted by length so a passing voxel stops early; the test
// |o|^2 / dta^2 + (de - dr)^2 / norm^2 <= 1 is taken as
// (de - dr)^2 <= (1 - |o|^2 / dta^2) norm^2.  counts[0] evaluated, counts[1]
// passed.
__global__ void __launch_bounds__(256) k_gamma(const double* ref, const double* ev, int nx,
                                               int ny, int nz, const double4* off, int n_off,
                                               double dd, double thr_abs, double max_ref,
                                               int local, unsigned long long* counts) {
    const size_t nvox = (size_t)nx * ny * nz;
    unsigned long long ne = 0, np = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvox;
         i += (size_t)gridDim.x * blockDim.x) {
        const double dr = ref[i];
        if (!(dr >= thr_abs) || dr <= 0.0) continue;
        ne++;
        const int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((size_t)nx * ny));
        const double norm = dd * (local ? dr : max_ref);
        const double norm2 = norm * norm;
        bool pass = false;
        for (int k = 0; k < n_off && !pass; ++k) {
            const double4 o = off[k];
            const double fx = ix + o.x, fy = iy + o.y, fz = iz + o.z;
            if (fx < 0.0 || fy < 0.0 || fz < 0.0 || fx > nx - 1 || fy > ny - 1 || fz > nz - 1)
                continue;
            int x0 = (int)floor(fx), y0 = (int)floor(fy), z0 = (int)floor(fz);
            if (x0 > nx - 2) x0 = nx > 1 ? nx - 2 : 0;
            if (y0 > ny - 2) y0 = ny > 1 ? ny - 2 : 0;
            if (z0 > nz - 2) z0 = nz > 1 ? nz - 2 : 0;
            const double tx = fx - x0, ty = fy - y0, tz = fz - z0;
            const int x1 = nx > 1 ? x0 + 1 : x0, y1 = ny > 1 ? y0 + 1 : y0, z1 = nz > 1 ? z0 + 1 : z0;
            const double* p00 = ev + ((size_t)z0 * ny + y0) * nx;
            const double* p10 = ev + ((size_t)z0 * ny + y1) * nx;
            const double* p01 = ev + ((size_t)z1 * ny + y0) * nx;
            const double* p11 = ev + ((size_t)z1 * ny + y1) * nx;
            const double c00 = p00[x0] * (1 - tx) + p00[x1] * tx;
            const double c10 = p10[x0] * (1 - tx) + p10[x1] * tx;
            const double c01 = p01[x0] * (1 - tx) + p01[x1] * tx;
            const double c11 = p11[x0] * (1 - tx) + p11[x1] * tx;
            const double c0 = c00 * (1 - ty) + c10 * ty, c1 = c01 * (1 - ty) + c11 * ty;
            const double diff = c0 * (1 - tz) + c1 * tz - dr;
            if (diff * diff <= (1.0 - o.w) * norm2) pass = true;
        }
        np += pass ? 1ull : 0ull;
    }
    ne = wave_sum64(ne);
    np = wave_sum64(np);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&counts[0], ne);
        atomicAdd(&counts[1], np);
    }
}

// Maximum of a non-negative double array via its bit pattern.
__global__ void k_max(const double* a, size_t n, unsigned long long* out) {
    double m = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        m = fmax(m, a[i]);
    unsigned long long b = (unsigned long long)__double_as_longlong(m);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long c = __shfl_xor(b, o);
        b = c > b ? c : b;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, b);
}

int blocks_for(size_t n, int block, int cap) {
    size_t g = (n + block - 1) / block;
    if (g > (size_t)cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t launch_gamma(const double* ref, const double* ev, int nx, int ny, int nz,
                        const double4* offsets, int n_off, double dd, double thr_abs,
                        double max_ref, int local, unsigned long long* counts, hipStream_t s) {
    const size_t nvox = (size_t)nx * ny * nz;
    hipLaunchKernelGGL(k_gamma, dim3(blocks_for(nvox, 256, 65536)), dim3(256), 0, s, ref, ev, nx,
                       ny, nz, offsets, n_off, dd, thr_abs, max_ref, local, counts);
    return hipGetLastError();
}

hipError_t launch_max(const double* a, size_t n, unsigned long long* out_bits, hipStream_t s) {
    // a grid-stride pass over few blocks: one same-address atomic per wave
    hipLaunchKernelGGL(k_max, dim3(blocks_for(n, 256, 1024)), dim3(256), 0, s, a, n, out_bits);
    return hipGetLastError();
}

}  // namespace sde

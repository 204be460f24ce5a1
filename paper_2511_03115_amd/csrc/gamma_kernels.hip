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

// Trilinear value of grid g at (fx, fy, fz) in voxel units; false outside
// [0, n - 1] on an axis.  The expression and the order of its operations are
// those of the definition, with no fused multiply-adds, so that the pass
// decision below is the same, bit for bit, as a double-precision evaluation
// of the definition.
__device__ __forceinline__ bool trilinear(const double* g, int nx, int ny, int nz, double fx,
                                          double fy, double fz, double& v) {
#pragma clang fp contract(off)
    if (fx < 0.0 || fy < 0.0 || fz < 0.0 || fx > nx - 1 || fy > ny - 1 || fz > nz - 1)
        return false;
    int x0 = (int)floor(fx), y0 = (int)floor(fy), z0 = (int)floor(fz);
    if (x0 > nx - 2) x0 = nx > 1 ? nx - 2 : 0;
    if (y0 > ny - 2) y0 = ny > 1 ? ny - 2 : 0;
    if (z0 > nz - 2) z0 = nz > 1 ? nz - 2 : 0;
    const double tx = fx - x0, ty = fy - y0, tz = fz - z0;
    const int x1 = nx > 1 ? x0 + 1 : x0, y1 = ny > 1 ? y0 + 1 : y0, z1 = nz > 1 ? z0 + 1 : z0;
    const double* p00 = g + ((size_t)z0 * ny + y0) * nx;
    const double* p10 = g + ((size_t)z0 * ny + y1) * nx;
    const double* p01 = g + ((size_t)z1 * ny + y0) * nx;
    const double* p11 = g + ((size_t)z1 * ny + y1) * nx;
    const double c00 = p00[x0] * (1 - tx) + p00[x1] * tx;
    const double c10 = p10[x0] * (1 - tx) + p10[x1] * tx;
    const double c01 = p01[x0] * (1 - tx) + p01[x1] * tx;
    const double c11 = p11[x0] * (1 - tx) + p11[x1] * tx;
    const double c0 = c00 * (1 - ty) + c10 * ty, c1 = c01 * (1 - ty) + c11 * ty;
    v = c0 * (1 - tz) + c1 * tz;
    return true;
}

// Range [lo, hi] of the trilinear interpolant of g over the box
// |x - node| <= r per axis around grid node (ix, iy, iz), clipped to the
// grid, for r <= 1 voxel on every axis.  The box then lies in the 8 cells
// around the node, the interpolant is multilinear in each, and so its
// extremes over the box are at the 27 points node + {-r, 0, r}^3 (clipped),
// evaluated here separably from the 27 node values around the node.
__device__ __forceinline__ void box_range(const double* g, int nx, int ny, int nz, int ix, int iy,
                                          int iz, double rx, double ry, double rz, double& lo,
                                          double& hi) {
    int xs[3] = {max(ix - 1, 0), ix, min(ix + 1, nx - 1)};
    int ys[3] = {max(iy - 1, 0), iy, min(iy + 1, ny - 1)};
    int zs[3] = {max(iz - 1, 0), iz, min(iz + 1, nz - 1)};
    double a[3][3][3];   // [z node][y node][x point]
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double* row = g + ((size_t)zs[k] * ny + ys[j]) * nx;
            const double v0 = row[xs[0]], v1 = row[xs[1]], v2 = row[xs[2]];
            a[k][j][0] = v1 + rx * (v0 - v1);
            a[k][j][1] = v1;
            a[k][j][2] = v1 + rx * (v2 - v1);
        }
    double b[3][3][3];   // [z node][y point][x point]
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const double v0 = a[k][0][p], v1 = a[k][1][p], v2 = a[k][2][p];
            b[k][0][p] = v1 + ry * (v0 - v1);
            b[k][1][p] = v1;
            b[k][2][p] = v1 + ry * (v2 - v1);
        }
    lo = b[1][1][1];
    hi = lo;
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const double v0 = b[0][q][p], v1 = b[1][q][p], v2 = b[2][q][p];
            const double m0 = v1 + rz * (v0 - v1), m2 = v1 + rz * (v2 - v1);
            lo = fmin(lo, fmin(v1, fmin(m0, m2)));
            hi = fmax(hi, fmax(v1, fmax(m0, m2)));
        }
}

// Gamma index, one thread per reference voxel.  off[k] = (ox / dx, oy / dy,
// oz / dz, |o|^2 / dta^2) for the lattice offsets o of spacing dta/interp
// within dta, nearest first (off[0] = 0); a voxel passes when
// |o|^2 / dta^2 + (de - dr)^2 / norm^2 <= 1 at some offset, de the trilinear
// value of the evaluated map there.  Voxels failing at o = 0 take a bound
// first (when dta is at most a voxel on every axis): every de reachable lies
// in the range of the interpolant over the search box, so with d the
// distance from dr to that range no offset passes once |o|^2 / dta^2 >
// 1 - d^2 / norm^2, and none at all when d > norm.  The bound is loosened by
// 1e-12 (relative in d, absolute in the limit) so that it never drops an
// offset whose evaluated test would pass.  counts[0] evaluated, counts[1]
// passed.
__global__ void __launch_bounds__(256) k_gamma(const double* ref, const double* ev, int nx,
                                               int ny, int nz, const double4* off, int n_off,
                                               double dd, double thr_abs, double max_ref,
                                               int local, double rx, double ry, double rz,
                                               int use_bound, unsigned long long* counts) {
#pragma clang fp contract(off)
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
        double de;
        if (trilinear(ev, nx, ny, nz, ix + off[0].x, iy + off[0].y, iz + off[0].z, de))
            pass = off[0].w + (de - dr) * (de - dr) / norm2 <= 1.0;
        double wmax = 2.0;   // offsets with |o|^2 / dta^2 above this cannot pass
        if (!pass && use_bound) {
            double lo, hi;
            box_range(ev, nx, ny, nz, ix, iy, iz, rx, ry, rz, lo, hi);
            const double d = dr < lo ? lo - dr : (dr > hi ? dr - hi : 0.0);
            const double ds = d - 1e-12 * fmax(fabs(dr), fmax(fabs(lo), fabs(hi)));
            if (ds > 0.0) wmax = 1.0 + 1e-12 - (ds * ds / norm2) * (1.0 - 1e-12);
        }
        for (int k = 1; k < n_off && !pass; ++k) {
            const double4 o = off[k];
            if (o.w > wmax) break;
            if (!trilinear(ev, nx, ny, nz, ix + o.x, iy + o.y, iz + o.z, de)) continue;
            if (o.w + (de - dr) * (de - dr) / norm2 <= 1.0) pass = true;
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

// Zero a few counters (a kernel, not a memset node, so the sequence can be
// captured in a graph).
__global__ void k_zero_u64(unsigned long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
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
                        double max_ref, int local, double rx, double ry, double rz, int use_bound,
                        unsigned long long* counts, hipStream_t s) {
    const size_t nvox = (size_t)nx * ny * nz;
    hipLaunchKernelGGL(k_gamma, dim3(blocks_for(nvox, 256, 65536)), dim3(256), 0, s, ref, ev, nx,
                       ny, nz, offsets, n_off, dd, thr_abs, max_ref, local, rx, ry, rz, use_bound,
                       counts);
    return hipGetLastError();
}

hipError_t launch_max(const double* a, size_t n, unsigned long long* out_bits, hipStream_t s) {
    // a grid-stride pass over few blocks: one same-address atomic per wave
    hipLaunchKernelGGL(k_max, dim3(blocks_for(n, 256, 1024)), dim3(256), 0, s, a, n, out_bits);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace sde

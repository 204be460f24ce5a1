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

constexpr int kMaxK = 50;   // largest interp (offsets per dta per axis)

// Everything the two gamma kernels read.
struct GammaArgs {
    const double* ref;
    const double* ev;
    int nx, ny, nz, K;
    double st, dta, dx, dy, dz;      // lattice spacing dta / K, dta, voxel size (cm)
    double dd, thr_abs, max_ref;
    int local, use_bound;
};

// Per axis and lattice index a in [-K, K]: a st (cm) and a st / d (voxels),
// in LDS.
struct GammaLattice {
    double cm[3][2 * kMaxK + 1];
    double vx[3][2 * kMaxK + 1];
};

__device__ __forceinline__ void fill_lattice(const GammaArgs& A, GammaLattice& L) {
    const int nl = 2 * A.K + 1;
    for (int t = threadIdx.x; t < 3 * nl; t += blockDim.x) {
        const int ax = t / nl, a = t % nl - A.K;
        const double v = a * A.st;
        L.cm[ax][a + A.K] = v;
        L.vx[ax][a + A.K] = v / (ax == 0 ? A.dx : ax == 1 ? A.dy : A.dz);
    }
    __syncthreads();
}

// The gamma test of reference voxel (ix, iy, iz) with dose dr at every
// offset but the zero one: the voxel passes when some offset o of the
// lattice of spacing st = dta/K within dta (o = st (a, b, c),
// a^2 + b^2 + c^2 <= K^2) has |o|^2 / dta^2 + (de - dr)^2 / norm^2 <= 1, de
// the trilinear value of the evaluated map at the voxel plus o.
//
// The lattice is walked octant by octant: with dta below a voxel on every
// axis, the offsets of one sign pattern all fall in one cell of the grid,
// whose 8 corner values are then held in registers and the trilinear value
// is formed factor by factor (the x factors once per a, the y factors once
// per b), the same products and sums in the same order as the definition's
// expression.  Per octant a bound first: the interpolant is multilinear in
// the cell, so its range over the octant's box is that of the box's 8
// corners; with d the distance from dr to the range, no offset with
// |o|^2 / dta^2 > 1 - d^2 / norm^2 passes, which limits a^2 + b^2 + c^2
// (loosened by 1e-9 so that no offset whose evaluated test would pass is
// dropped).  Each offset's test is screened with multiplications by
// reciprocals; within 1e-12 of the boundary it is decided by the
// definition's divisions, so the decision is the same, bit for bit, as a
// double-precision evaluation of the definition.  An offset whose cell is
// not the octant's (dta at or above a voxel, or rounding at a face) takes the
// general evaluation.
__device__ bool gamma_search(const GammaArgs& A, const GammaLattice& L, int ix, int iy, int iz,
                             double dr) {
#pragma clang fp contract(off)
    const int nx = A.nx, ny = A.ny, nz = A.nz, K = A.K, KK = K * K;
    const double* ev = A.ev;
    const double dta = A.dta, inv_dta2 = 1.0 / (dta * dta);
    const double norm = A.dd * (A.local ? dr : A.max_ref);
    const double norm2 = norm * norm, inv_n2 = 1.0 / norm2;
    for (int oct = 0; oct < 8; ++oct) {
        // sign pattern: s = 0 takes a >= 0 (cell [i, i+1]), s = 1 takes a < 0 (cell [i-1, i])
        const int sx = oct & 1, sy = (oct >> 1) & 1, sz = oct >> 2;
        if ((sx && ix == 0) || (sy && iy == 0) || (sz && iz == 0)) continue;   // outside
        int x0 = ix - sx, y0 = iy - sy, z0 = iz - sz;
        if (x0 > nx - 2) x0 = nx > 1 ? nx - 2 : 0;
        if (y0 > ny - 2) y0 = ny > 1 ? ny - 2 : 0;
        if (z0 > nz - 2) z0 = nz > 1 ? nz - 2 : 0;
        const int x1 = nx > 1 ? x0 + 1 : x0, y1 = ny > 1 ? y0 + 1 : y0, z1 = nz > 1 ? z0 + 1 : z0;
        const double* p00 = ev + ((size_t)z0 * ny + y0) * nx;
        const double* p10 = ev + ((size_t)z0 * ny + y1) * nx;
        const double* p01 = ev + ((size_t)z1 * ny + y0) * nx;
        const double* p11 = ev + ((size_t)z1 * ny + y1) * nx;
        const double v000 = p00[x0], v100 = p00[x1], v010 = p10[x0], v110 = p10[x1];
        const double v001 = p01[x0], v101 = p01[x1], v011 = p11[x0], v111 = p11[x1];
        int nmax = KK;
        if (A.use_bound) {
            // the octant's box in cell coordinates, its corners, the range
            const double rx = L.vx[0][2 * K], ry = L.vx[1][2 * K], rz = L.vx[2][2 * K];
            const double ax0 = sx ? 1.0 - rx : (double)(ix - x0),
                         ax1 = sx ? 1.0 : fmin((double)(ix - x0) + rx, 1.0);
            const double ay0 = sy ? 1.0 - ry : (double)(iy - y0),
                         ay1 = sy ? 1.0 : fmin((double)(iy - y0) + ry, 1.0);
            const double az0 = sz ? 1.0 - rz : (double)(iz - z0),
                         az1 = sz ? 1.0 : fmin((double)(iz - z0) + rz, 1.0);
            double lo = 1e300, hi = -1e300;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const double tx = (c & 1) ? ax1 : ax0, ty = (c & 2) ? ay1 : ay0,
                             tz = (c & 4) ? az1 : az0;
                const double e00 = v000 + tx * (v100 - v000), e10 = v010 + tx * (v110 - v010);
                const double e01 = v001 + tx * (v101 - v001), e11 = v011 + tx * (v111 - v011);
                const double e0 = e00 + ty * (e10 - e00), e1 = e01 + ty * (e11 - e01);
                const double e = e0 + tz * (e1 - e0);
                lo = fmin(lo, e);
                hi = fmax(hi, e);
            }
            const double d = dr < lo ? lo - dr : (dr > hi ? dr - hi : 0.0);
            const double ds = d - 1e-12 * fmax(fabs(dr), fmax(fabs(lo), fabs(hi)));
            if (ds > 0.0) {
                const double wmax = 1.0 - ds * ds * inv_n2;   // |o|^2 / dta^2 at most
                if (wmax < 0.0) continue;                    // the octant cannot pass
                nmax = min(KK, (int)(wmax * KK * (1.0 + 1e-9)) + 1);
            }
        }
        // a in [0, K] (s = 0) or [-K, -1] (s = 1), walked outward
        for (int ua = 0; ua + sx <= K; ++ua) {
            const int a = sx ? -(ua + 1) : ua;
            if (a * a > nmax) break;
            const double fx = ix + L.vx[0][a + K];
            if (fx < 0.0 || fx > nx - 1) continue;
            int xf = (int)floor(fx);
            if (xf > nx - 2) xf = nx > 1 ? nx - 2 : 0;
            const bool xin = xf == x0;
            const double tx = fx - x0;
            const double c00 = v000 * (1 - tx) + v100 * tx, c10 = v010 * (1 - tx) + v110 * tx;
            const double c01 = v001 * (1 - tx) + v101 * tx, c11 = v011 * (1 - tx) + v111 * tx;
            const double oxx = L.cm[0][a + K] * L.cm[0][a + K];
            for (int ub = 0; ub + sy <= K; ++ub) {
                const int b = sy ? -(ub + 1) : ub;
                if (a * a + b * b > nmax) break;
                const double fy = iy + L.vx[1][b + K];
                if (fy < 0.0 || fy > ny - 1) continue;
                int yf = (int)floor(fy);
                if (yf > ny - 2) yf = ny > 1 ? ny - 2 : 0;
                const bool yin = yf == y0;
                const double ty = fy - y0;
                const double c0 = c00 * (1 - ty) + c10 * ty, c1 = c01 * (1 - ty) + c11 * ty;
                const double sab = oxx + L.cm[1][b + K] * L.cm[1][b + K];
                if (A.use_bound && xin && yin) {
                    // Along the row the offsets stay in the octant's cell, where
                    // v - dr = al + be c is linear in c, so the test function
                    // sab/dta^2 + c^2 st^2/dta^2 + (al + be c)^2/norm^2 is a
                    // convex quadratic in c: its continuous minimum bounds every
                    // offset of the row, and above 1 (by a margin far beyond
                    // rounding) no offset of the row passes.
                    const double t0 = (double)(iz - z0), h = L.vx[2][K + 1];
                    const double al = (c0 + (c1 - c0) * t0) - dr, be = (c1 - c0) * h;
                    const double qa = L.cm[2][K + 1] * L.cm[2][K + 1] * inv_dta2;
                    const double qb = be * be * inv_n2;
                    const double cs = -(al * be * inv_n2) / (qa + qb);
                    const double lin = al + be * cs;
                    const double fmin = sab * inv_dta2 + qa * cs * cs + lin * lin * inv_n2;
                    if (fmin > 1.0 + 1e-9) continue;
                }
                for (int uc = 0; uc + sz <= K; ++uc) {
                    const int c = sz ? -(uc + 1) : uc;
                    if (a * a + b * b + c * c > nmax) break;
                    if (a == 0 && b == 0 && c == 0) continue;   // the zero offset: tested apart
                    const double fz = iz + L.vx[2][c + K];
                    if (fz < 0.0 || fz > nz - 1) continue;
                    int zf = (int)floor(fz);
                    if (zf > nz - 2) zf = nz > 1 ? nz - 2 : 0;
                    double v;
                    if (xin && yin && zf == z0) {
                        const double tz = fz - z0;
                        v = c0 * (1 - tz) + c1 * tz;
                    } else if (!trilinear(ev, nx, ny, nz, fx, fy, fz, v)) {
                        continue;
                    }
                    const double r2 = sab + L.cm[2][c + K] * L.cm[2][c + K];
                    const double diff = v - dr;
                    const double gf = r2 * inv_dta2 + diff * diff * inv_n2;
                    if (gf > 1.0 + 1e-12) continue;
                    if (gf < 1.0 - 1e-12 || r2 / (dta * dta) + diff * diff / norm2 <= 1.0)
                        return true;
                }
            }
        }
    }
    return false;
}

// Pass 1 of the gamma index, one thread per reference voxel: the
// threshold, then the zero offset (|o|^2 / dta^2 = 0 / dta^2).  A voxel
// failing there is appended to the list of voxels to search (one atomic
// per wave); beyond the list's capacity it is searched at once.
// counts = {evaluated, passed, (maximum), list length}.
__global__ void __launch_bounds__(256) k_gamma_screen(GammaArgs A, unsigned long long* counts,
                                                      unsigned* list, unsigned cap) {
#pragma clang fp contract(off)
    __shared__ GammaLattice L;
    fill_lattice(A, L);
    const int nx = A.nx, ny = A.ny, nz = A.nz, K = A.K;
    const size_t nvox = (size_t)nx * ny * nz;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    unsigned long long ne = 0, np = 0;
    // the loop runs a whole number of rounds per wave so the ballot sees every lane
    for (size_t i0 = blockIdx.x * (size_t)blockDim.x + (threadIdx.x & ~63u); i0 < nvox;
         i0 += stride) {
        const size_t i = i0 + lane;
        bool hard = false;
        int ix = 0, iy = 0, iz = 0;
        double dr = 0.0;
        if (i < nvox) {
            dr = A.ref[i];
            if (dr >= A.thr_abs && dr > 0.0) {
                ne++;
                ix = (int)(i % nx);
                iy = (int)((i / nx) % ny);
                iz = (int)(i / ((size_t)nx * ny));
                const double norm = A.dd * (A.local ? dr : A.max_ref);
                double de;
                bool pass = false;
                if (trilinear(A.ev, nx, ny, nz, ix + L.vx[0][K], iy + L.vx[1][K],
                              iz + L.vx[2][K], de))
                    pass = (L.cm[0][K] * L.cm[0][K] + L.cm[1][K] * L.cm[1][K] +
                            L.cm[2][K] * L.cm[2][K]) / (A.dta * A.dta) +
                               (de - dr) * (de - dr) / (norm * norm) <= 1.0;
                if (pass) np++;
                else hard = true;
            }
        }
        const unsigned long long m = __ballot(hard);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(&counts[3], (unsigned long long)__popcll(m));
            base = __shfl(base, leader);
            if (hard) {
                const unsigned long long slot = base + __popcll(m & ((1ull << lane) - 1ull));
                if (slot < cap) list[slot] = (unsigned)i;
                else if (gamma_search(A, L, ix, iy, iz, dr)) np++;
            }
        }
    }
    // same-address atomics serialise in L2: one per wave, and none for a
    // wave that evaluated nothing (most of a dose map is below threshold)
    ne = wave_sum64(ne);
    np = wave_sum64(np);
    if (lane == 0 && ne) {
        atomicAdd(&counts[0], ne);
        if (np) atomicAdd(&counts[1], np);
    }
}

// Pass 2: the listed voxels, one thread each, so that the waves doing the
// long searches are full.
__global__ void __launch_bounds__(256) k_gamma_search(GammaArgs A, unsigned long long* counts,
                                                      const unsigned* list, unsigned cap) {
    __shared__ GammaLattice L;
    fill_lattice(A, L);
    const unsigned long long nl = counts[3] < cap ? counts[3] : cap;
    unsigned long long np = 0;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < nl;
         k += (size_t)gridDim.x * blockDim.x) {
        const size_t i = list[k];
        const int ix = (int)(i % A.nx), iy = (int)((i / A.nx) % A.ny),
                  iz = (int)(i / ((size_t)A.nx * A.ny));
        if (gamma_search(A, L, ix, iy, iz, A.ref[i])) np++;
    }
    np = wave_sum64(np);
    if ((threadIdx.x & 63) == 0 && np) atomicAdd(&counts[1], np);
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

hipError_t launch_gamma(const double* ref, const double* ev, int nx, int ny, int nz, int interp,
                        double dta, double dx, double dy, double dz, double dd, double thr_abs,
                        double max_ref, int local, int use_bound, unsigned long long* counts,
                        unsigned* list, unsigned cap, hipStream_t s) {
    if (interp < 1 || interp > kMaxK) return hipErrorInvalidValue;
    const size_t nvox = (size_t)nx * ny * nz;
    GammaArgs A{ref, ev, nx, ny, nz, interp, dta / interp, dta, dx, dy, dz, dd, thr_abs, max_ref,
                local, use_bound};
    // a grid-stride pass over at most 4096 workgroups keeps the counter
    // atomics few (one per wave that evaluated something)
    hipLaunchKernelGGL(k_gamma_screen, dim3(blocks_for(nvox, 256, 4096)), dim3(256), 0, s, A,
                       counts, list, cap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the list's length is on the device: a grid that covers a large list,
    // grid-stride beyond
    hipLaunchKernelGGL(k_gamma_search, dim3(blocks_for(cap, 256, 8192)), dim3(256), 0, s, A,
                       counts, list, cap);
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

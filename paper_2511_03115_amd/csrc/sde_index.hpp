// Index arithmetic of the transport kernel, shared with a CPU build that
// checks it: the voxel of a position, the linear voxel index, the slot of a
// voxel in the workgroup's LDS tile, and the energy-lattice interval.
//
// Built with -DSDE_CHECKS (on the host only), every result is checked
// against the bounds its caller relies on and a violation aborts with the
// offending values; without it the checks compile to nothing.
#pragma once

#include <hip/hip_runtime.h>

#ifdef SDE_CHECKS
#include <cstdio>
#include <cstdlib>
#define SDE_CHECK(cond, fmt, ...)                                                  \
    do {                                                                           \
        if (!(cond)) {                                                             \
            std::fprintf(stderr, "SDE_CHECKS: %s: " fmt "\n", #cond, __VA_ARGS__); \
            std::abort();                                                          \
        }                                                                          \
    } while (0)
#else
#define SDE_CHECK(cond, fmt, ...) ((void)0)
#endif

namespace sde {

// Voxel along one axis of a point with lo <= x <= hi (the box's closed
// extent): floor((x - lo) / d), the upper face belonging to the last voxel.
// float multiplies by the reciprocal voxel size, double divides.
__host__ __device__ inline int axis_voxel(float x, float lo, float inv_d, float, int n) {
    const int c = (int)((x - lo) * inv_d), i = c < n - 1 ? c : n - 1;
    SDE_CHECK(i >= 0 && i < n, "x=%.9g lo=%.9g inv_d=%.9g n=%d i=%d", (double)x, (double)lo,
              (double)inv_d, n, i);
    return i;
}
__host__ __device__ inline int axis_voxel(double x, double lo, double, double d, int n) {
    const int c = (int)((x - lo) / d), i = c < n - 1 ? c : n - 1;
    SDE_CHECK(i >= 0 && i < n, "x=%.17g lo=%.17g d=%.17g n=%d i=%d", x, lo, d, n, i);
    return i;
}

// Linear index (iz ny + iy) nx + ix of an in-range voxel, in 32 bits
// (phantoms have fewer than 2^31 voxels).
__host__ __device__ inline int voxel_index(int ix, int iy, int iz, int nx, int ny, int nz) {
    SDE_CHECK(ix >= 0 && ix < nx && iy >= 0 && iy < ny && iz >= 0 && iz < nz &&
                  (long long)nx * ny * nz < (1ll << 31),
              "(%d %d %d) of (%d %d %d)", ix, iy, iz, nx, ny, nz);
    return (int)(((unsigned)iz * (unsigned)ny + (unsigned)iy) * (unsigned)nx + (unsigned)ix);
}

// Slot of voxel (ix, iy, iz) in the tile [x0, x0 + tnx) x ... (-1 outside).
__host__ __device__ inline int tile_slot(int ix, int iy, int iz, int x0, int y0, int z0, int tnx,
                                         int tny, int tnz) {
    const unsigned tx = (unsigned)(ix - x0), ty = (unsigned)(iy - y0), tz = (unsigned)(iz - z0);
    if (!(tx < (unsigned)tnx && ty < (unsigned)tny && tz < (unsigned)tnz)) return -1;
    const int s = (int)((tz * (unsigned)tny + ty) * (unsigned)tnx + tx);
    SDE_CHECK(s >= 0 && s < tnx * tny * tnz, "slot %d of %d", s, tnx * tny * tnz);
    return s;
}

// Lattice interval i in [0, n_e - 2] of lattice coordinate t (rows i and
// i + 1 are read).
__host__ __device__ inline int lattice_interval(float t, int n_e) {
    const int c = (int)t, i = c < 0 ? 0 : (c > n_e - 2 ? n_e - 2 : c);
    SDE_CHECK(i >= 0 && i + 1 < n_e, "t=%.9g n_e=%d i=%d", (double)t, n_e, i);
    return i;
}
__host__ __device__ inline int lattice_interval(double t, int n_e) {
    const int c = (int)t, i = c < 0 ? 0 : (c > n_e - 2 ? n_e - 2 : c);
    SDE_CHECK(i >= 0 && i + 1 < n_e, "t=%.17g n_e=%d i=%d", t, n_e, i);
    return i;
}

}  // namespace sde

// The transport kernel's index arithmetic (paper_2511_03115_amd/csrc/
// sde_index.hpp) built on the CPU with -DSDE_CHECKS (bounds checked) and the
// sanitizers, driven with the kernel's own float arithmetic over the phantom
// geometries of the workloads and odd ones:
//  * every inside point maps to an in-range voxel, at most one voxel from
//    floor((x - lo) / d) in exact arithmetic;
//  * a step's midpoint fma(o, Delta/2, r) lies inside the box whenever its
//    start r and end fma(o, Delta, r) do (the kernel scores it unchecked);
//  * the linear voxel index stays below the voxel count;
//  * a voxel's LDS tile slot is in range exactly when the voxel is in the
//    tile, and distinct voxels get distinct slots;
//  * the energy-lattice interval is in range for every float energy in
//    [e_min, e_max] and just outside it.
// With the argument "plant", one out-of-box point is passed on purpose and
// the run must abort with an SDE_CHECKS message.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "sde_index.hpp"

using namespace sde;

static int failures = 0;
#define EXPECT(c, ...)                              \
    do {                                                 \
        if (!(c)) {                                      \
            if (failures++ < 20) std::printf(__VA_ARGS__); \
        }                                                \
    } while (0)

struct Box {
    int n[3];
    double d[3], origin[3];
};

// the float box as the host fills the kernel's scalars
struct FBox {
    float lo[3], hi[3], inv_d[3];
    explicit FBox(const Box& b) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = (float)b.origin[a];
            hi[a] = (float)(b.origin[a] + b.n[a] * b.d[a]);
            inv_d[a] = (float)(1.0 / b.d[a]);
        }
    }
    bool inside(float x, float y, float z) const {
        return x >= lo[0] && x <= hi[0] && y >= lo[1] && y <= hi[1] && z >= lo[2] && z <= hi[2];
    }
};

static void check_box(const Box& b, std::mt19937_64& rng) {
    const FBox F(b);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    // axis voxels: random points, faces and their float neighbours
    for (int a = 0; a < 3; ++a) {
        std::vector<float> xs = {F.lo[a], F.hi[a], std::nextafter(F.lo[a], F.hi[a]),
                                 std::nextafter(F.hi[a], F.lo[a])};
        for (int k = 0; k <= b.n[a]; ++k) {   // voxel faces and their neighbours
            const float f = (float)(b.origin[a] + k * b.d[a]);
            for (float x : {f, std::nextafter(f, -1e30f), std::nextafter(f, 1e30f)})
                if (x >= F.lo[a] && x <= F.hi[a]) xs.push_back(x);
        }
        for (int k = 0; k < 20000; ++k)
            xs.push_back((float)(F.lo[a] + U(rng) * ((double)F.hi[a] - F.lo[a])));
        for (float x : xs) {
            if (!(x >= F.lo[a] && x <= F.hi[a])) continue;
            const int i = axis_voxel(x, F.lo[a], F.inv_d[a], 0.0f, b.n[a]);
            const double exact = std::floor(((double)x - b.origin[a]) / b.d[a]);
            const int ie = (int)std::min<double>(std::max(exact, 0.0), b.n[a] - 1);
            EXPECT(std::abs(i - ie) <= 1, "axis %d x=%.9g voxel %d exact %d\n", a, (double)x, i, ie);
            const int i64 = axis_voxel((double)x, b.origin[a], 0.0, b.d[a], b.n[a]);
            EXPECT(i64 == ie, "axis %d x=%.9g double voxel %d exact %d\n", a, (double)x, i64, ie);
        }
    }
    // steps: start inside, end inside => midpoint inside; voxel index range
    const float step = 0.05f, half = 0.5f * step;
    const long long nvox = (long long)b.n[0] * b.n[1] * b.n[2];
    std::normal_distribution<double> N(0.0, 1.0);
    for (int k = 0; k < 400000; ++k) {
        float r[3], o[3];
        const bool near_face = k % 2;
        for (int a = 0; a < 3; ++a) {
            double t = U(rng);
            if (near_face) t = (k / 2) % 3 == a ? (U(rng) < 0.5 ? U(rng) * 1e-4 : 1 - U(rng) * 1e-4) : t;
            r[a] = (float)(F.lo[a] + t * ((double)F.hi[a] - F.lo[a]));
            r[a] = std::fmin(std::fmax(r[a], F.lo[a]), F.hi[a]);
        }
        double g[3] = {N(rng), N(rng), N(rng)};
        const double gn = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        for (int a = 0; a < 3; ++a) o[a] = (float)(g[a] / gn);
        if (k % 7 == 0) { o[0] = 0.0f; o[1] = 0.0f; o[2] = (k % 14) ? 1.0f : -1.0f; }
        float nx[3], m[3];
        for (int a = 0; a < 3; ++a) {
            nx[a] = std::fma(o[a], step, r[a]);
            m[a] = std::fma(o[a], half, r[a]);
        }
        if (!F.inside(r[0], r[1], r[2]) || !F.inside(nx[0], nx[1], nx[2])) continue;
        EXPECT(F.inside(m[0], m[1], m[2]), "midpoint outside: r=(%.9g %.9g %.9g) o=(%.9g %.9g %.9g)\n",
               (double)r[0], (double)r[1], (double)r[2], (double)o[0], (double)o[1], (double)o[2]);
        const int ix = axis_voxel(m[0], F.lo[0], F.inv_d[0], 0.0f, b.n[0]);
        const int iy = axis_voxel(m[1], F.lo[1], F.inv_d[1], 0.0f, b.n[1]);
        const int iz = axis_voxel(m[2], F.lo[2], F.inv_d[2], 0.0f, b.n[2]);
        const int v = voxel_index(ix, iy, iz, b.n[0], b.n[1], b.n[2]);
        EXPECT(v >= 0 && v < nvox, "voxel index %d of %lld\n", v, nvox);
    }
}

static void check_tile(int tnx, int tny, int tnz, int x0, int y0, int z0, const Box& b) {
    std::vector<char> seen((size_t)tnx * tny * tnz, 0);
    for (int iz = 0; iz < b.n[2]; iz += (b.n[2] > 64 ? 3 : 1))
        for (int iy = 0; iy < b.n[1]; ++iy)
            for (int ix = 0; ix < b.n[0]; ++ix) {
                const int s = tile_slot(ix, iy, iz, x0, y0, z0, tnx, tny, tnz);
                const bool in = ix >= x0 && ix < x0 + tnx && iy >= y0 && iy < y0 + tny &&
                                iz >= z0 && iz < z0 + tnz;
                EXPECT((s >= 0) == in, "tile membership (%d %d %d)\n", ix, iy, iz);
                if (s >= 0) {
                    EXPECT(s < tnx * tny * tnz, "slot %d\n", s);
                    EXPECT(!seen[s], "slot %d taken twice\n", s);
                    seen[s] = 1;
                }
            }
}

static void check_lattice(double e_min, double e_max, int n_e) {
    const double ln_lo = std::log(e_min), dln = (std::log(e_max) - ln_lo) / (n_e - 1);
    const float ln_lo_f = (float)ln_lo, inv_f = (float)(1.0 / dln);
    const double inv_d = 1.0 / dln;
    std::vector<float> Es;
    for (float E = (float)e_min * 0.999f; E <= (float)e_max * 1.001f; E *= 1.0007f) Es.push_back(E);
    Es.push_back((float)e_min);
    Es.push_back((float)e_max);
    for (float E : Es) {
        const float tl = (std::log(E) - ln_lo_f) * inv_f;
        const int i = lattice_interval(tl, n_e);
        EXPECT(i >= 0 && i + 1 < n_e, "lattice E=%.9g i=%d\n", (double)E, i);
        const int i64 = lattice_interval((std::log((double)E) - ln_lo) * inv_d, n_e);
        EXPECT(i64 >= 0 && i64 + 1 < n_e, "lattice (double) E=%.9g i=%d\n", (double)E, i64);
    }
}

int main(int argc, char** argv) {
    if (argc > 1 && std::strcmp(argv[1], "plant") == 0) {
        // a point below the box: the check must fire
        const int i = axis_voxel(-1.0f, 0.0f, 10.0f, 0.0f, 100);
        std::printf("not caught: %d\n", i);
        return 0;
    }
    std::mt19937_64 rng(12345);
    const Box boxes[] = {
        {{200, 200, 300}, {0.1, 0.1, 0.1}, {-10.0, -10.0, 0.0}},      // water, 1 mm
        {{200, 200, 200}, {0.1, 0.1, 0.1}, {-10.0, -10.0, 0.0}},      // slab / insert / CT
        {{256, 256, 200}, {0.2, 0.2, 0.2}, {-25.6, -25.6, 0.0}},      // plan, 2 mm
        {{37, 41, 53}, {0.123, 0.0917, 0.3}, {-2.2755, 1.5, -7.0}},    // odd sizes and origins
        {{1, 1, 1}, {100.0, 100.0, 5.0}, {-50.0, -50.0, 0.0}},        // one voxel
    };
    for (const Box& b : boxes) check_box(b, rng);
    const Box small = {{40, 30, 50}, {0.1, 0.1, 0.1}, {0, 0, 0}};
    check_tile(8, 8, 20, 16, 11, 0, small);
    check_tile(40, 30, 50, 0, 0, 0, small);      // the whole phantom
    check_tile(1, 1, 1, 39, 29, 49, small);      // the last voxel
    check_tile(8, 8, 20, 36, 26, 40, small);     // reaching past the phantom
    check_lattice(0.05, 260.0, 1024);
    check_lattice(0.05, 260.0, 16);
    check_lattice(1.0, 300.0, 4096);
    std::printf("%s: %d failures\n", failures ? "FAILED" : "done", failures);
    return failures ? 1 : 0;
}

// The C ABI's host-side validation (sde_api.cpp with sde_tables.cpp) under
// AddressSanitizer and UndefinedBehaviorSanitizer, on a host without a GPU:
// every entry point refuses bad arguments before any device call, and a
// valid sde_init_materials fails cleanly when no device is present.  The
// kernel launchers are replaced by stubs that report "not supported" (no
// path exercised here reaches them).  Exits non-zero on an unexpected code.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "inputs.hpp"
#include "sde.h"
#include "sde_internal.hpp"

namespace sde {
hipError_t launch_pack_phantom(const uint8_t*, const float*, uint2*, size_t, int, unsigned int*,
                               unsigned int*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_reset(unsigned long long*, size_t, unsigned long long*, unsigned long long*,
                        hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_transport(const KParams&, int, int, size_t, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_convert(unsigned long long*, int, const uint2*, size_t, double, double, double*,
                          unsigned long long*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_gamma(const double*, const double*, int, int, int, int, double, double, double,
                        double, double, double, double, int, int, unsigned long long*, unsigned*,
                        unsigned, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_zero_u64(unsigned long long*, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_max(const double*, size_t, unsigned long long*, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_sbm_polar(const float*, const float*, const float*, int, float*, float*,
                            hipStream_t) { return hipErrorNotSupported; }
hipError_t transport_kernel_attributes(size_t) { return hipErrorNotSupported; }
hipError_t launch_philox_words(unsigned long long, const unsigned long long*, const unsigned*,
                               const unsigned*, int, uint4*, hipStream_t) {
    return hipErrorNotSupported;
}
}  // namespace sde

static int failures = 0;

static void expect(const char* what, int rc, int want) {
    const bool ok = rc == want;
    std::printf("%-58s rc=%d want=%d %s  [%s]\n", what, rc, want, ok ? "ok" : "UNEXPECTED",
                sde_last_error());
    if (!ok) ++failures;
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    const Bundle b = Bundle::read(argv[1]);
    Inputs in(b);

    expect("sde_last_error starts empty", (int)std::strlen(sde_last_error()), 0);
    // transport and plans before the tables
    sde_spot spot{};
    spot.E_MeV = 100;
    spot.n_histories = 10;
    spot.weight = 1;
    sde_beam beam{};
    beam.n_spots = 1;
    beam.spots = &spot;
    std::vector<uint8_t> mat(8, 0);
    std::vector<float> rho(8, 1.0f);
    sde_phantom ph{};
    ph.nx = ph.ny = ph.nz = 2;
    ph.dx_cm = ph.dy_cm = ph.dz_cm = 0.1;
    ph.material_id = mat.data();
    ph.density = rho.data();
    std::vector<double> dose(8);
    expect("transport before init", sde_transport(&beam, &ph, 10, 1, dose.data()), SDE_E_STATE);
    expect("transport with NULL dose", sde_transport(&beam, &ph, 10, 1, nullptr), SDE_E_INVALID);
    sde_plan* plan = nullptr;
    expect("plan before init", sde_plan_create(&beam, &ph, 10, 1, nullptr, &plan), SDE_E_STATE);
    expect("plan with NULL out", sde_plan_create(&beam, &ph, 10, 1, nullptr, nullptr), SDE_E_INVALID);
    expect("plan_execute NULL", sde_plan_execute(nullptr, dose.data(), 0), SDE_E_INVALID);
    expect("plan_destroy NULL", sde_plan_destroy(nullptr), SDE_OK);

    // tables: refused before any device call
    expect("init: no materials", sde_init_materials(nullptr, 0, &in.params, nullptr), SDE_E_INVALID);
    sde_physics_params bad = in.params;
    bad.step_cm = -1;
    expect("init: negative step",
           sde_init_materials(in.mats.data(), (int)in.mats.size(), &bad, &in.nuc), SDE_E_INVALID);
    bad = in.params;
    bad.flags |= 1024u;
    expect("init: unknown switch",
           sde_init_materials(in.mats.data(), (int)in.mats.size(), &bad, &in.nuc), SDE_E_INVALID);
    sde_nuclear_tables nb = in.nuc;
    nb.n_l = 12;
    expect("init: 12 partial waves",
           sde_init_materials(in.mats.data(), (int)in.mats.size(), &in.params, &nb), SDE_E_INVALID);

    // test entry points: argument checks first
    float f4[4] = {0};
    expect("sbm_polar n < 0", sde_sbm_polar(f4, f4, f4, -1, f4, f4), SDE_E_INVALID);
    expect("sbm_polar NULL", sde_sbm_polar(nullptr, f4, f4, 4, f4, f4), SDE_E_INVALID);
    expect("sbm_polar n = 0", sde_sbm_polar(nullptr, nullptr, nullptr, 0, nullptr, nullptr), SDE_OK);
    alignas(16) uint32_t words[8];
    uint64_t h[2] = {1, 2};
    uint32_t n2[2] = {0, 1}, b2[2] = {0, 0};
    expect("philox count < 0", sde_philox_words(1, h, n2, b2, -1, words), SDE_E_INVALID);
    expect("philox NULL", sde_philox_words(1, nullptr, n2, b2, 2, words), SDE_E_INVALID);
    expect("philox misaligned", sde_philox_words(1, h, n2, b2, 2, words + 1), SDE_E_INVALID);
    expect("philox count 0", sde_philox_words(1, nullptr, nullptr, nullptr, 0, nullptr), SDE_OK);
    int64_t counts[2];
    std::vector<double> map(27, 1.0);
    auto gam = [&](int nx, double dx, double dd, double dta, double thr, int interp, int64_t* c,
                   const double* r) {
        return sde_gamma(r, map.data(), nx, 3, 3, dx, 0.1, 0.1, dd, dta, thr, interp, 0, c);
    };
    expect("gamma NULL reference", gam(3, 0.1, 0.01, 0.05, 0.1, 10, counts, nullptr), SDE_E_INVALID);
    expect("gamma NULL counts", gam(3, 0.1, 0.01, 0.05, 0.1, 10, nullptr, map.data()), SDE_E_INVALID);
    expect("gamma nx 0", gam(0, 0.1, 0.01, 0.05, 0.1, 10, counts, map.data()), SDE_E_INVALID);
    expect("gamma voxel size 0", gam(3, 0.0, 0.01, 0.05, 0.1, 10, counts, map.data()), SDE_E_INVALID);
    expect("gamma dd 0", gam(3, 0.1, 0.0, 0.05, 0.1, 10, counts, map.data()), SDE_E_INVALID);
    expect("gamma dta NaN", gam(3, 0.1, 0.01, std::nan(""), 0.1, 10, counts, map.data()),
           SDE_E_INVALID);
    expect("gamma interp 0", gam(3, 0.1, 0.01, 0.05, 0.1, 0, counts, map.data()), SDE_E_INVALID);
    expect("gamma interp 51", gam(3, 0.1, 0.01, 0.05, 0.1, 51, counts, map.data()), SDE_E_INVALID);
    expect("gamma_noalloc NULL", sde_gamma_noalloc(nullptr, map.data(), 3, 3, 3, 0.1, 0.1, 0.1,
                                                   0.01, 0.05, 0.1, 10, 0, counts),
           SDE_E_INVALID);

    // a valid table build reaches the device: without one, a clean error
    const int rc = sde_init_materials(in.mats.data(), (int)in.mats.size(), &in.params, &in.nuc);
    std::printf("init without a device: rc=%d [%s]\n", rc, sde_last_error());
    if (rc == SDE_OK) ++failures;   // there is no GPU here
    expect("transport after a failed init", sde_transport(&beam, &ph, 10, 1, dose.data()),
           SDE_E_STATE);
    sde_free();
    sde_free();
    std::printf("%s: %d unexpected\n", failures ? "FAILED" : "done", failures);
    return failures ? 1 : 0;
}

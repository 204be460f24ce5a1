// Host-side table bundle of libsde (built by sde_tables.cpp, uploaded by sde_api.cpp).
#pragma once

#include <string>
#include <vector>

#include "sde.h"
#include "sde_internal.hpp"

namespace sde {

struct HostTables {
    int n_mat = 0, n_e = 0, n_u = 2, n_tab = 0;
    double e_lo = 0, e_hi = 0, ln_e_lo = 0, dln = 0;
    std::vector<float4> hot;
    std::vector<double2> rg64;
    std::vector<MatDev> mats;
    std::vector<float> nuc_sigma, nuc_u, nuc_r, nuc_a;
    // the FP64 instance's copies
    std::vector<MatDev64> mats64;
    std::vector<double2> hot64;
    std::vector<double> nuc_sigma64, nuc_u64, nuc_r64, nuc_a64;
    // elastic nuclear data
    int n_ni = 0, n_mu = 0, n_l = 0;
    std::vector<float> ni_p, ni_cum, ni_sig;
    std::vector<double> ni_p64, ni_cum64, ni_sig64, h_coef;
    double ruth_T = 0, mott_lo = 0, mott_hi = 0, mott_D0 = 0, mott_Lhi = 0, mott_Llo = 0;
    double mott_Dlo = 0, mott_shi = 0, mott_slo = 0;
    double c_strag = 0;
    sde_physics_params params{};
};

int build_host_tables(const sde_material_desc* mats, int n_mats, const sde_physics_params* p,
                      const sde_nuclear_tables* nuc, HostTables* out, std::string* err);

}  // namespace sde

// Reader of the input bundle written by tests/test_sanitizers.py: named
// arrays of float64 or int32, so that the sanitized drivers take the same
// materials, physics parameters and nuclear tables (inelastic and elastic)
// as the rest of the test suite.
//
// File: "SDEIN1" then records {char name[32]; int32 kind (0 f64, 1 i32);
// int64 count; count elements}.
#pragma once

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "sde.h"

struct Bundle {
    std::map<std::string, std::vector<double>> f;
    std::map<std::string, std::vector<int>> i;

    static Bundle read(const char* path) {
        Bundle b;
        FILE* fp = std::fopen(path, "rb");
        if (!fp) { std::fprintf(stderr, "cannot open %s\n", path); std::exit(2); }
        char magic[6];
        if (std::fread(magic, 1, 6, fp) != 6 || std::memcmp(magic, "SDEIN1", 6) != 0) {
            std::fprintf(stderr, "bad bundle\n");
            std::exit(2);
        }
        for (;;) {
            char name[33] = {0};
            int32_t kind;
            int64_t n;
            if (std::fread(name, 1, 32, fp) != 32) break;
            if (std::fread(&kind, 4, 1, fp) != 1 || std::fread(&n, 8, 1, fp) != 1 || n < 0) {
                std::fprintf(stderr, "truncated bundle\n");
                std::exit(2);
            }
            if (kind == 0) {
                std::vector<double> v((size_t)n);
                if (n && std::fread(v.data(), 8, (size_t)n, fp) != (size_t)n) std::exit(2);
                b.f[name] = std::move(v);
            } else {
                std::vector<int> v((size_t)n);
                if (n && std::fread(v.data(), 4, (size_t)n, fp) != (size_t)n) std::exit(2);
                b.i[name] = std::move(v);
            }
        }
        std::fclose(fp);
        return b;
    }
    const std::vector<double>& F(const std::string& k) const {
        auto it = f.find(k);
        if (it == f.end()) { std::fprintf(stderr, "missing %s\n", k.c_str()); std::exit(2); }
        return it->second;
    }
    const std::vector<int>& I(const std::string& k) const {
        auto it = i.find(k);
        if (it == i.end()) { std::fprintf(stderr, "missing %s\n", k.c_str()); std::exit(2); }
        return it->second;
    }
};

// The C-ABI descriptors over a bundle's arrays (which must outlive them).
struct Inputs {
    std::vector<sde_material_desc> mats;
    sde_physics_params params{};
    sde_nuclear_tables nuc{};

    explicit Inputs(const Bundle& b) {
        const int n_mat = b.I("n_mat")[0];
        for (int k = 0; k < n_mat; ++k) {
            const std::string p = "mat" + std::to_string(k);
            sde_material_desc d{};
            d.n_elem = (int)b.I(p + ".Z").size();
            d.Z = b.I(p + ".Z").data();
            d.A = b.F(p + ".A").data();
            d.w = b.F(p + ".w").data();
            d.I_eV = b.F(p + ".I")[0];
            mats.push_back(d);
        }
        const auto& pp = b.F("params");
        params.step_cm = pp[0];
        params.ld_z_cm = pp[1];
        params.e_min_MeV = pp[2];
        params.e_max_MeV = pp[3];
        params.ld_F = pp[4];
        params.theta_cut_rad = pp[5];
        params.backscatter_cut_rad = pp[6];
        params.max_steps = (int64_t)pp[7];
        params.n_energy = b.I("params.n_energy")[0];
        params.flags = (unsigned)b.I("params.flags")[0];
        const auto& c = b.I("nuc.counts");   // n_tab, n_u, n_ni, n_mu, n_l
        nuc.n_tab = c[0];
        nuc.n_u = c[1];
        nuc.Z = b.I("nuc.Z").data();
        nuc.sigma_barn = b.F("nuc.sigma").data();
        nuc.u_icdf = b.F("nuc.u_icdf").data();
        nuc.kalbach_r = b.F("nuc.kr").data();
        nuc.kalbach_a = b.F("nuc.ka").data();
        nuc.n_ni = c[2];
        nuc.n_mu = c[3];
        nuc.ni_Z = b.I("nuc.ni_Z").data();
        nuc.ni_sigma_barn = b.F("nuc.ni_sigma").data();
        nuc.ni_p = b.F("nuc.ni_p").data();
        nuc.n_l = c[4];
        nuc.h_a_re = b.F("nuc.h_are").data();
        nuc.h_a_im = b.F("nuc.h_aim").data();
        nuc.h_b = b.F("nuc.h_b").data();
    }
};

// The host table build of libsde (sde_tables.cpp) under AddressSanitizer
// and UndefinedBehaviorSanitizer: every physics-switch combination with and
// without nuclear data, then inputs that must be refused.  Prints one line
// per case; exits non-zero on an unexpected return code (the sanitizers
// abort on their own findings).
#include <cmath>
#include <cstdio>
#include <limits>
#include <string>
#include <vector>

#include "inputs.hpp"
#include "sde_host.hpp"

using sde::HostTables;

static int failures = 0;

static double checksum(const HostTables& T) {
    double s = 0;
    for (const auto& h : T.hot) s += h.x + h.y + h.z + h.w;
    for (const auto& r : T.rg64) s += r.x + r.y;
    for (const auto& h : T.hot64) s += h.x + h.y;
    for (double c : T.ni_cum64) s += c;
    for (double c : T.h_coef) s += c;
    return s;
}

static void expect(const char* what, int rc, int want, const std::string& err) {
    const bool ok = want == SDE_OK ? rc == SDE_OK : rc != SDE_OK;
    std::printf("%-52s rc=%d %s%s\n", what, rc, ok ? "ok" : "UNEXPECTED",
                err.empty() ? "" : (" (" + err + ")").c_str());
    if (!ok) ++failures;
}

static int build(const Inputs& in, const sde_physics_params& p, const sde_nuclear_tables* nuc,
                 std::string* err, double* sum = nullptr) {
    HostTables T;
    err->clear();
    const int rc = sde::build_host_tables(in.mats.data(), (int)in.mats.size(), &p, nuc, &T, err);
    if (rc == SDE_OK && sum) *sum = checksum(T);
    return rc;
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    const Bundle b = Bundle::read(argv[1]);
    const Inputs in(b);
    const double nan = std::numeric_limits<double>::quiet_NaN();
    std::string err;

    // valid: every combination of the switch groups, with and without data
    const unsigned sets[] = {SDE_ALL, SDE_ALL | SDE_FP64, SDE_ALL | SDE_ECUT,
                             SDE_ALL | SDE_ECUT | SDE_FP64, SDE_LOSS, SDE_LOSS | SDE_ELASTIC,
                             SDE_LOSS | SDE_INELASTIC | SDE_END_OF_RANGE, 0u};
    for (unsigned f : sets) {
        for (int with : {0, 1, 2}) {   // no data, inelastic only, inelastic + elastic
            sde_physics_params p = in.params;
            p.flags = f;
            sde_nuclear_tables n = in.nuc;
            if (with == 1) n.n_ni = n.n_l = 0;
            double sum = 0;
            const int rc = build(in, p, with ? &n : nullptr, &err, &sum);
            char what[96];
            std::snprintf(what, sizeof what, "flags %u, nuclear data %d", f, with);
            expect(what, rc, SDE_OK, err);
            if (rc == SDE_OK && !std::isfinite(sum)) {
                std::printf("  non-finite table\n");
                ++failures;
            }
        }
    }

    // parameters that must be refused
    struct PCase {
        const char* what;
        void (*edit)(sde_physics_params&);
    };
    const PCase pcases[] = {
        {"step 0", [](sde_physics_params& p) { p.step_cm = 0; }},
        {"step NaN", [](sde_physics_params& p) { p.step_cm = std::nan(""); }},
        {"z negative", [](sde_physics_params& p) { p.ld_z_cm = -1; }},
        {"e_min 0", [](sde_physics_params& p) { p.e_min_MeV = 0; }},
        {"e_max <= e_min", [](sde_physics_params& p) { p.e_max_MeV = p.e_min_MeV; }},
        {"n_energy 15", [](sde_physics_params& p) { p.n_energy = 15; }},
        {"F 1", [](sde_physics_params& p) { p.ld_F = 1; }},
        {"cut pi", [](sde_physics_params& p) { p.theta_cut_rad = M_PI; }},
        {"backscatter cut 0", [](sde_physics_params& p) { p.backscatter_cut_rad = 0; }},
        {"max_steps 0", [](sde_physics_params& p) { p.max_steps = 0; }},
        {"unknown switch bit", [](sde_physics_params& p) { p.flags |= 512u; }},
    };
    for (const auto& c : pcases) {
        sde_physics_params p = in.params;
        c.edit(p);
        expect(c.what, build(in, p, &in.nuc, &err), SDE_E_INVALID, err);
    }

    // materials that must be refused
    {
        HostTables T;
        err.clear();
        expect("no materials", sde::build_host_tables(in.mats.data(), 0, &in.params, nullptr, &T, &err),
               SDE_E_INVALID, err);
        std::vector<sde_material_desc> many(9, in.mats[0]);
        err.clear();
        expect("nine materials", sde::build_host_tables(many.data(), 9, &in.params, nullptr, &T, &err),
               SDE_E_INVALID, err);
    }
    auto mat_case = [&](const char* what, auto edit) {
        std::vector<sde_material_desc> m = in.mats;
        std::vector<int> Z(m[0].Z, m[0].Z + m[0].n_elem);
        std::vector<double> A(m[0].A, m[0].A + m[0].n_elem), w(m[0].w, m[0].w + m[0].n_elem);
        edit(m[0], Z, A, w);
        m[0].Z = Z.data();
        m[0].A = A.data();
        m[0].w = w.data();
        HostTables T;
        err.clear();
        expect(what, sde::build_host_tables(m.data(), (int)m.size(), &in.params, &in.nuc, &T, &err),
               SDE_E_INVALID, err);
    };
    mat_case("n_elem 0", [](sde_material_desc& d, auto&, auto&, auto&) { d.n_elem = 0; });
    mat_case("n_elem 17", [](sde_material_desc& d, auto&, auto&, auto&) { d.n_elem = 17; });
    mat_case("Z 0", [](sde_material_desc&, std::vector<int>& Z, auto&, auto&) { Z[0] = 0; });
    mat_case("Z 101", [](sde_material_desc&, std::vector<int>& Z, auto&, auto&) { Z[0] = 101; });
    mat_case("A NaN", [&](sde_material_desc&, auto&, std::vector<double>& A, auto&) { A[0] = nan; });
    mat_case("w negative", [](sde_material_desc&, auto&, auto&, std::vector<double>& w) { w[0] = -0.1; });
    mat_case("w NaN", [&](sde_material_desc&, auto&, auto&, std::vector<double>& w) { w[0] = nan; });
    mat_case("weights all zero", [](sde_material_desc&, auto&, auto&, std::vector<double>& w) {
        for (auto& x : w) x = 0;
    });
    mat_case("I 0", [](sde_material_desc& d, auto&, auto&, auto&) { d.I_eV = 0; });
    mat_case("I 5000 eV (negative stopping power)", [](sde_material_desc& d, auto&, auto&, auto&) {
        d.I_eV = 5000;
    });

    // nuclear tables that must be refused
    auto nuc_case = [&](const char* what, auto edit) {
        sde_nuclear_tables n = in.nuc;
        std::vector<double> sig(b.F("nuc.sigma")), u(b.F("nuc.u_icdf")), kr(b.F("nuc.kr")),
            ka(b.F("nuc.ka")), nis(b.F("nuc.ni_sigma")), nip(b.F("nuc.ni_p")), hb(b.F("nuc.h_b"));
        edit(n, sig, u, kr, ka, nis, nip, hb);
        n.sigma_barn = sig.data();
        n.u_icdf = u.data();
        n.kalbach_r = kr.data();
        n.kalbach_a = ka.data();
        n.ni_sigma_barn = nis.data();
        n.ni_p = nip.data();
        n.h_b = hb.data();
        expect(what, build(in, in.params, &n, &err), SDE_E_INVALID, err);
    };
    using V = std::vector<double>;
    nuc_case("n_u 1", [](sde_nuclear_tables& n, V&, V&, V&, V&, V&, V&, V&) { n.n_u = 1; });
    nuc_case("n_tab 65", [](sde_nuclear_tables& n, V&, V&, V&, V&, V&, V&, V&) { n.n_tab = 65; });
    nuc_case("sigma negative", [](sde_nuclear_tables&, V& s, V&, V&, V&, V&, V&, V&) { s[3] = -1; });
    nuc_case("sigma NaN", [&](sde_nuclear_tables&, V& s, V&, V&, V&, V&, V&, V&) { s[5] = nan; });
    nuc_case("u icdf NaN", [&](sde_nuclear_tables&, V&, V& u, V&, V&, V&, V&, V&) { u[7] = nan; });
    nuc_case("u icdf decreasing", [](sde_nuclear_tables&, V&, V& u, V&, V&, V&, V&, V&) {
        u[1] = u[2] + 0.5;
    });
    nuc_case("u icdf above 1", [](sde_nuclear_tables&, V&, V& u, V&, V&, V&, V&, V&) {
        u[2] = 1.5;
    });
    nuc_case("Kalbach r above 1", [](sde_nuclear_tables&, V&, V&, V& r, V&, V&, V&, V&) { r[0] = 2; });
    nuc_case("Kalbach a negative", [](sde_nuclear_tables&, V&, V&, V&, V& a, V&, V&, V&) { a[0] = -1; });
    nuc_case("Kalbach a NaN", [&](sde_nuclear_tables&, V&, V&, V&, V& a, V&, V&, V&) { a[4] = nan; });
    nuc_case("n_mu 6", [](sde_nuclear_tables& n, V&, V&, V&, V&, V&, V&, V&) { n.n_mu = 6; });
    nuc_case("n_mu 257", [](sde_nuclear_tables& n, V&, V&, V&, V&, V&, V&, V&) { n.n_mu = 257; });
    nuc_case("n_l 9", [](sde_nuclear_tables& n, V&, V&, V&, V&, V&, V&, V&) { n.n_l = 9; });
    nuc_case("n_ni 65", [](sde_nuclear_tables& n, V&, V&, V&, V&, V&, V&, V&) { n.n_ni = 65; });
    nuc_case("sigma_NI negative", [](sde_nuclear_tables&, V&, V&, V&, V&, V& s, V&, V&) { s[1] = -1; });
    nuc_case("P_NI NaN", [&](sde_nuclear_tables&, V&, V&, V&, V&, V&, V& p, V&) { p[9] = nan; });
    nuc_case("h b NaN", [&](sde_nuclear_tables&, V&, V&, V&, V&, V&, V&, V& h) { h[2] = nan; });

    std::printf("%s: %d unexpected\n", failures ? "FAILED" : "done", failures);
    return failures ? 1 : 0;
}

// Host-side FP64 table generation for libsde.
//
// For every medium, on the lattice of n_energy points uniform in ln E over
// [e_min, e_max]:
//   hot[i]  = {A1, A2, ne, el} (FP32, staged in LDS by the transport kernel)
//     A1 = chi_c^2/rho / (1 + F^2) * Delta / z     (per unit density)
//     A2 = chi_c^2/rho / (2 chi_alpha^2 (1 - F))   (so nu = rho A2)
//     so that the per-step polar width is sigma^2 = rho A1 ((1+nu)/nu ln(1+nu) - 1),
//     the Lynch-Dahl width of section 2.1.4 scaled to the step;
//     ne = inelastic jump rate per unit density (piecewise linear on the
//          lattice by definition, so linear interpolation is exact);
//     el = elastic jump rate per unit density times E^2: the Rutherford part
//          is constant and the Mott part nearly so, so interpolating el and
//          dividing by E^2 keeps the rate's 1/E^2 shape exact;
//   rg64[i] = {Rg, dRg/dt} in FP64 for the cubic-Hermite end-of-range decision;
//   hot64[i] = {ne, el} unrounded, and per medium the Lynch-Dahl, Bethe and
//   jump constants in FP64 (MatDev64), for the double-precision instance.
// Per element: the constants of the rate laws (section 2.1.4, Eq.
// (large_elastic_cm) and Eq. (large_elastic_cm_hydrogen); section 2.1.5).
#include <cmath>
#include <string>
#include <vector>

#include "sde.h"
#include "sde_elastic.hpp"
#include "sde_host.hpp"
#include "sde_internal.hpp"

namespace sde {

namespace {

struct Medium {
    int n;
    double Z[kMaxElem], A[kMaxElem], w[kMaxElem];
    double I_MeV;
};

double zoa(const Medium& m) {
    double s = 0;
    for (int i = 0; i < m.n; ++i) s += m.w[i] * m.Z[i] / m.A[i];
    return s;
}

// Mass stopping power (MeV cm^2/g), Eq. (bethbloch) with Bragg additivity.
double stopping(const Medium& m, double E) {
    const double g = E + kMp;
    const double p2 = E * (E + 2.0 * kMp);
    const double b2 = p2 / (g * g);
    const double L = std::log(2.0 * kMe * p2 / (kMp * kMp) / m.I_MeV) - b2;
    return kBethe * zoa(m) / b2 * L;
}

// Gauss-Legendre rule of order 12 by Newton iteration on P_12.
struct Gauss {
    double x[12], w[12];
    Gauss() {
        const int n = 12;
        for (int i = 0; i < n; ++i) {
            double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), d = 1.0;
            for (int it = 0; it < 60; ++it) {
                double a = 1.0, b = z;
                for (int k = 2; k <= n; ++k) {
                    const double c = ((2.0 * k - 1.0) * z * b - (k - 1.0) * a) / k;
                    a = b;
                    b = c;
                }
                d = n * (z * b - a) / (z * z - 1.0);
                const double dz = b / d;
                z -= dz;
                if (std::fabs(dz) < 1e-15) break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * d * d);
        }
    }
};

// int_{E0}^{E1} dE / S = int E/S d(ln E), Gauss-Legendre in ln E.
double range_piece(const Medium& m, const Gauss& G, double E0, double E1) {
    const double a = std::log(E0), b = std::log(E1);
    const double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double s = 0;
    for (int k = 0; k < 12; ++k) {
        const double E = std::exp(c + h * G.x[k]);
        s += G.w[k] * E / stopping(m, E);
    }
    return s * h;
}

// Lynch-Dahl chi_c^2 per unit density and chi_alpha^2 (section 2.1.4).
void lynch_dahl(const Medium& m, double E, double z, double& chic2_per_rho, double& chia2) {
    const double p2 = E * (E + 2.0 * kMp);
    const double pb = p2 / (E + kMp);
    const double b2 = p2 / ((E + kMp) * (E + kMp));
    double c = 0, num = 0, den = 0;
    for (int i = 0; i < m.n; ++i) {
        const double Z = m.Z[i];
        const double wz = m.w[i] * Z * (Z + 1.0) / m.A[i];
        c += 0.157 * wz * z / (pb * pb);
        const double za = Z * kAlpha;
        num += wz * std::log(2.007e-5 * std::cbrt(Z * Z) * (1.0 + 3.34 * za * za / b2) / p2);
        den += wz;
    }
    chic2_per_rho = c;
    chia2 = std::exp(num / den);
}

}  // namespace

// Build all tables; returns SDE_OK or an error code with a message.
int build_host_tables(const sde_material_desc* mats, int n_mats, const sde_physics_params* p,
                      const sde_nuclear_tables* nuc, HostTables* out, std::string* err) {
    if (!mats || n_mats < 1 || n_mats > kMaxMat) {
        *err = "n_mats must be in 1..8";
        return SDE_E_INVALID;
    }
    if (!p || !(p->step_cm > 0) || !(p->ld_z_cm > 0) || !(p->e_min_MeV > 0) ||
        !(p->e_max_MeV > p->e_min_MeV) || p->n_energy < 16 || !(p->ld_F > 0 && p->ld_F < 1) ||
        !(p->theta_cut_rad > 0 && p->theta_cut_rad < M_PI) ||
        !(p->backscatter_cut_rad > 0 && p->backscatter_cut_rad < M_PI) || p->max_steps < 1) {
        *err = "invalid physics parameters";
        return SDE_E_INVALID;
    }
    if (p->flags & ~(unsigned)(SDE_ALL | SDE_FP64 | SDE_ECUT)) {
        *err = "unknown physics switch bits";
        return SDE_E_INVALID;
    }
    HostTables& T = *out;
    T = HostTables();
    T.params = *p;
    T.n_mat = n_mats;
    T.n_e = p->n_energy;
    T.e_lo = p->e_min_MeV;
    T.e_hi = p->e_max_MeV;
    T.ln_e_lo = std::log(T.e_lo);
    T.dln = (std::log(T.e_hi) - T.ln_e_lo) / (T.n_e - 1);
    const double ahc = kAlpha * kHbarcFm;                 // MeV fm
    const double ahc_cm = ahc * 1e-13;
    T.c_strag = 4.0 * M_PI * kNa * ahc_cm * ahc_cm;        // MeV^2 cm^2 / mol
    // angular limits of the large-angle laws
    const double omc = 2.0 * std::pow(std::sin(0.5 * p->theta_cut_rad), 2);   // 1 - cos
    T.ruth_T = 1.0 / omc;
    T.mott_hi = std::cos(p->theta_cut_rad);
    T.mott_lo = -std::cos(p->backscatter_cut_rad);
    {
        const double s_hi = std::sin(p->theta_cut_rad), s_lo = std::sin(p->backscatter_cut_rad);
        T.mott_D0 = 2.0 * T.mott_hi / (s_hi * s_hi) - 2.0 * T.mott_lo / (s_lo * s_lo);
        T.mott_Dlo = 2.0 * T.mott_lo / (s_lo * s_lo);
        T.mott_shi = omc;
        T.mott_slo = 1.0 + std::cos(p->backscatter_cut_rad);
        T.mott_Lhi = std::log((1.0 + T.mott_hi) / omc);
        const double omb = 2.0 * std::pow(std::sin(0.5 * p->backscatter_cut_rad), 2);
        T.mott_Llo = std::log(omb / (1.0 - T.mott_lo));
    }

    // nuclear tables
    const bool use_ne = nuc && nuc->n_tab > 0;
    if (use_ne) {
        if (!nuc->Z || !nuc->sigma_barn || !nuc->u_icdf || !nuc->kalbach_r || !nuc->kalbach_a ||
            nuc->n_u < 2 || nuc->n_tab > 64) {
            *err = "invalid nuclear tables";
            return SDE_E_INVALID;
        }
        T.n_tab = nuc->n_tab;
        T.n_u = nuc->n_u;
        const size_t ns = (size_t)T.n_tab * T.n_e, nu = ns * T.n_u;
        T.nuc_sigma.resize(ns);
        T.nuc_u.resize(nu);
        T.nuc_r.resize(nu);
        T.nuc_a.resize(nu);
        for (size_t i = 0; i < ns; ++i) {
            if (!(nuc->sigma_barn[i] >= 0) || !std::isfinite(nuc->sigma_barn[i])) {
                *err = "negative or non-finite cross section";
                return SDE_E_INVALID;
            }
            T.nuc_sigma[i] = (float)nuc->sigma_barn[i];
        }
        for (size_t i = 0; i < nu; ++i) {
            // the loss fraction's inverse CDF: in [0, 1], nondecreasing in U;
            // Kalbach-Mann r in [0, 1], a >= 0 (NaN fails every test)
            const double u = nuc->u_icdf[i], r = nuc->kalbach_r[i], a = nuc->kalbach_a[i];
            if (!(u >= 0 && u <= 1) || (i % T.n_u && !(u >= nuc->u_icdf[i - 1]))) {
                *err = "loss-fraction inverse CDF outside [0, 1] or decreasing";
                return SDE_E_INVALID;
            }
            if (!(r >= 0 && r <= 1) || !(a >= 0 && std::isfinite(a))) {
                *err = "Kalbach-Mann r outside [0, 1] or a negative";
                return SDE_E_INVALID;
            }
            T.nuc_u[i] = (float)u;
            T.nuc_r[i] = (float)r;
            T.nuc_a[i] = (float)a;
        }
        T.nuc_sigma64.assign(nuc->sigma_barn, nuc->sigma_barn + ns);
        T.nuc_u64.assign(nuc->u_icdf, nuc->u_icdf + nu);
        T.nuc_r64.assign(nuc->kalbach_r, nuc->kalbach_r + nu);
        T.nuc_a64.assign(nuc->kalbach_a, nuc->kalbach_a + nu);
    } else {
        T.nuc_sigma.assign(1, 0.f);
        T.nuc_u.assign(2, 0.f);
        T.nuc_r.assign(2, 0.f);
        T.nuc_a.assign(2, 0.f);
        T.nuc_sigma64.assign(1, 0.0);
        T.nuc_u64.assign(2, 0.0);
        T.nuc_r64.assign(2, 0.0);
        T.nuc_a64.assign(2, 0.0);
    }

    // elastic nuclear data (section 2.1.4)
    const bool use_ni = nuc && nuc->n_ni > 0, use_h = nuc && nuc->n_l > 0;
    if (nuc && (nuc->n_ni < 0 || nuc->n_ni > 64 || nuc->n_l < 0 || nuc->n_l > kMaxL ||
                (use_ni && (!nuc->ni_Z || !nuc->ni_sigma_barn || !nuc->ni_p || nuc->n_mu < 7 ||
                            nuc->n_mu > 256)) ||
                (use_h && (!nuc->h_a_re || !nuc->h_a_im || !nuc->h_b)))) {
        *err = "invalid elastic nuclear tables";
        return SDE_E_INVALID;
    }
    if (use_ni) {
        T.n_ni = nuc->n_ni;
        T.n_mu = nuc->n_mu;
        const int m = T.n_mu - 3;
        const double hk = 2.0 / m;
        const size_t nrow = (size_t)T.n_ni * T.n_e;
        T.ni_p64.assign(nuc->ni_p, nuc->ni_p + nrow * T.n_mu);
        T.ni_sig64.assign(nuc->ni_sigma_barn, nuc->ni_sigma_barn + nrow);
        T.ni_cum64.assign(nrow * (m + 1), 0.0);
        for (size_t i = 0; i < nrow * T.n_mu; ++i)
            if (!std::isfinite(T.ni_p64[i])) { *err = "non-finite P_NI coefficient"; return SDE_E_INVALID; }
        for (size_t r = 0; r < nrow; ++r) {
            if (!(T.ni_sig64[r] >= 0) || !std::isfinite(T.ni_sig64[r])) {
                *err = "negative or non-finite sigma_NI";
                return SDE_E_INVALID;
            }
            const double* c = &T.ni_p64[r * T.n_mu];
            double* cum = &T.ni_cum64[r * (m + 1)];
            for (int k = 0; k < m; ++k)   // a full knot interval: h (c_k + 11 c_k+1 + 11 c_k+2 + c_k+3) / 24
                cum[k + 1] = cum[k] + hk * (c[k] + 11.0 * c[k + 1] + 11.0 * c[k + 2] + c[k + 3]) / 24.0;
        }
        T.ni_p.assign(T.ni_p64.begin(), T.ni_p64.end());
        T.ni_cum.assign(T.ni_cum64.begin(), T.ni_cum64.end());
        T.ni_sig.assign(T.ni_sig64.begin(), T.ni_sig64.end());
    } else {
        T.ni_p.assign(1, 0.f);
        T.ni_cum.assign(1, 0.f);
        T.ni_sig.assign(1, 0.f);
        T.ni_p64.assign(1, 0.0);
        T.ni_cum64.assign(1, 0.0);
        T.ni_sig64.assign(1, 0.0);
    }
    if (use_h) {
        T.n_l = nuc->n_l;
        const size_t nc = (size_t)T.n_l * (T.n_e + 2);
        T.h_coef.resize(3 * nc);
        std::copy(nuc->h_a_re, nuc->h_a_re + nc, T.h_coef.begin());
        std::copy(nuc->h_a_im, nuc->h_a_im + nc, T.h_coef.begin() + nc);
        std::copy(nuc->h_b, nuc->h_b + nc, T.h_coef.begin() + 2 * nc);
        for (double c : T.h_coef)
            if (!std::isfinite(c)) { *err = "non-finite hydrogen amplitude"; return SDE_E_INVALID; }
    } else {
        T.h_coef.assign(1, 0.0);
    }
    // hydrogen amplitudes at lattice point i (the spline at an integer
    // lattice coordinate: (c_i + 4 c_i+1 + c_i+2) / 6)
    auto h_amp_at = [&](int i) {
        HAmp a{};
        a.n_l = T.n_l;
        const size_t nc = (size_t)T.n_l * (T.n_e + 2);
        for (int l = 0; l < T.n_l; ++l) {
            const double* c = &T.h_coef[(size_t)l * (T.n_e + 2) + i];
            a.are[l] = (c[0] + 4.0 * c[1] + c[2]) / 6.0;
            a.aim[l] = (c[nc] + 4.0 * c[nc + 1] + c[nc + 2]) / 6.0;
            a.b[l] = (c[2 * nc] + 4.0 * c[2 * nc + 1] + c[2 * nc + 2]) / 6.0;
        }
        return a;
    };

    const Gauss G;
    T.hot.resize((size_t)n_mats * T.n_e);
    T.hot64.resize((size_t)n_mats * T.n_e);
    T.rg64.resize((size_t)n_mats * T.n_e);
    T.mats.resize(n_mats);
    T.mats64.resize(n_mats);
    std::vector<double> E(T.n_e);
    for (int i = 0; i < T.n_e; ++i) E[i] = std::exp(T.ln_e_lo + i * T.dln);
    E[0] = T.e_lo;
    E[T.n_e - 1] = T.e_hi;

    for (int k = 0; k < n_mats; ++k) {
        const sde_material_desc& d = mats[k];
        if (d.n_elem < 1 || d.n_elem > kMaxElem || !d.Z || !d.A || !d.w || !(d.I_eV > 0)) {
            *err = "invalid material " + std::to_string(k);
            return SDE_E_INVALID;
        }
        Medium m{};
        m.n = d.n_elem;
        double wsum = 0;
        for (int i = 0; i < m.n; ++i) {
            if (d.Z[i] < 1 || d.Z[i] > 100 || !(d.A[i] > 0) || !(d.w[i] >= 0)) {
                *err = "invalid element in material " + std::to_string(k);
                return SDE_E_INVALID;
            }
            m.Z[i] = d.Z[i];
            m.A[i] = d.A[i];
            m.w[i] = d.w[i];
            wsum += d.w[i];
        }
        if (!(wsum > 0)) { *err = "mass fractions sum to zero"; return SDE_E_INVALID; }
        for (int i = 0; i < m.n; ++i) m.w[i] /= wsum;
        m.I_MeV = d.I_eV * 1e-6;
        if (!(stopping(m, T.e_lo) > 0)) {
            *err = "stopping power not positive at e_min for material " + std::to_string(k);
            return SDE_E_INVALID;
        }

        MatDev md{};
        MatDev64 m64{};
        double c_ruth_d = 0, c_mott_d = 0, c_ruth0_d = 0;   // FP64 sums of the elastic coefficients
        m64.zoa = zoa(m);
        m64.log_pre = std::log(2.0 * kMe / m.I_MeV) - 2.0 * std::log(kMp);
        m64.n_elem = m.n;
        md.zoa = (float)m64.zoa;
        md.log_pre = (float)m64.log_pre;
        md.n_elem = m.n;
        for (int i = 0; i < m.n; ++i) {
            ElemDev& e = md.el[i];
            const double Z = m.Z[i], A = m.A[i];
            const double nd = kNa * m.w[i] / A;                 // atoms per g
            const double ek = Z * ahc * (1.0 + A) / (2.0 * A);  // (eta/k) E, fm MeV
            e.Z = (float)Z;
            e.m2 = (float)(A * kAmu);
            e.is_h = (d.Z[i] == 1);
            // 2 pi (azimuth) x atoms/g x 1e-24 cm^2/barn x 0.01 barn/fm^2
            const double pre = 2.0 * M_PI * nd * 1e-24 * 0.01 * ek * ek;
            e.el_coef = (float)(e.is_h ? pre : pre * (T.ruth_T - 0.5));
            e.el_base = (float)pre;
            if (!e.is_h) c_ruth0_d += pre;
            e.ne_coef = (float)(nd * 1e-24);
            e.tab = -1;
            if (use_ne)
                for (int t = 0; t < nuc->n_tab; ++t)
                    if (nuc->Z[t] == d.Z[i]) e.tab = t;
            if (e.is_h) e.tab = -1;
            const double coef = e.is_h ? pre : pre * (T.ruth_T - 0.5);
            if (e.is_h) c_mott_d += coef; else c_ruth_d += coef;
            m64.wz[i] = m.w[i] * Z * (Z + 1.0) / A;
            m64.ln_ca[i] = std::log(2.007e-5 * std::cbrt(Z * Z));
            m64.za2[i] = 3.34 * (Z * kAlpha) * (Z * kAlpha);
            m64.el_coef[i] = coef;
            m64.el_base[i] = pre;
            m64.ne_coef[i] = nd * 1e-24;
            m64.m2[i] = A * kAmu;
            m64.is_h[i] = e.is_h;
            m64.tab[i] = e.tab;
            // elastic nuclear terms: rate / rho per barn of CM integral
            const double nuc_coef = 2.0 * M_PI * nd * 1e-24;
            e.nuc_coef = (float)nuc_coef;
            m64.nuc_coef[i] = nuc_coef;
            e.ni = -1;
            if (use_ni && !e.is_h)
                for (int t = 0; t < nuc->n_ni; ++t)
                    if (nuc->ni_Z[t] == d.Z[i]) e.ni = t;
            e.hn = (e.is_h && use_h) ? 1 : 0;
            m64.ni[i] = e.ni;
            m64.hn[i] = e.hn;
        }

        // elastic rate per unit density times E^2 at lattice point li (the
        // Coulomb parts, and the nuclear terms at the fixed cut)
        auto el_e2_at = [&](int li) {
            const double En = E[li];
            const double eta = kAlpha * std::sqrt(kMp / (2.0 * En));
            const double mott = T.mott_D0 - (std::sin(eta * T.mott_Lhi) -
                                             std::sin(eta * T.mott_Llo)) / (2.0 * eta);
            if (!(p->flags & SDE_ELASTIC)) return 0.0;
            double r = c_ruth_d + c_mott_d * mott, nucl = 0.0;
            for (int i = 0; i < m.n; ++i) {
                const ElemDev& e = md.el[i];
                if (e.ni >= 0) {
                    const size_t row = (size_t)e.ni * T.n_e + li;
                    double dens, integ;
                    ni_spline(&T.ni_p64[row * T.n_mu], &T.ni_cum64[row * (T.n_mu - 2)],
                              T.n_mu - 3, T.mott_hi, dens, integ);
                    nucl += m64.nuc_coef[i] * T.ni_sig64[row] * integ;
                } else if (e.hn) {
                    const HAmp a = h_amp_at(li);
                    double d0, d1, g0, g1;
                    h_nuclear(a, eta, T.mott_hi, d1, g1);
                    h_nuclear(a, eta, T.mott_lo, d0, g0);
                    nucl += m64.nuc_coef[i] * (g1 - g0);
                }
            }
            return r + nucl * En * En;
        };
        // inelastic rate per unit density at lattice point li
        auto ne_rate_at = [&](int li) {
            double r = 0;
            for (int i = 0; i < m.n; ++i) {
                const ElemDev& e = md.el[i];
                if ((p->flags & SDE_INELASTIC) && e.tab >= 0)
                    r += kNa * m.w[i] / m.A[i] * 1e-24 *
                         nuc->sigma_barn[(size_t)e.tab * T.n_e + li];
            }
            return r;
        };

        double Rg = 0;
        const double Fp = p->ld_F;
        for (int i = 0; i < T.n_e; ++i) {
            if (i > 0) Rg += range_piece(m, G, E[i - 1], E[i]);
            double c2, ca2;
            lynch_dahl(m, E[i], p->ld_z_cm, c2, ca2);
            float4 h;
            h.x = (float)(c2 / (1.0 + Fp * Fp) * p->step_cm / p->ld_z_cm);
            h.y = (float)(c2 / (2.0 * ca2 * (1.0 - Fp)));
            h.z = (float)ne_rate_at(i);
            const double el_e2 = el_e2_at(i);
            h.w = (float)el_e2;
            T.hot[(size_t)k * T.n_e + i] = h;
            T.hot64[(size_t)k * T.n_e + i] = make_double2(ne_rate_at(i), el_e2);
            double2 r;
            r.x = Rg;
            r.y = E[i] / stopping(m, E[i]) * T.dln;   // dRg / dt, t the lattice coordinate
            T.rg64[(size_t)k * T.n_e + i] = r;
        }
        md.c_ruth = (float)c_ruth_d;
        md.c_mott = (float)c_mott_d;
        md.c_ruth0 = (float)c_ruth0_d;
        T.mats[k] = md;
        m64.c_ruth = c_ruth_d;
        m64.c_mott = c_mott_d;
        m64.c_ruth0 = c_ruth0_d;
        T.mats64[k] = m64;
    }
    return SDE_OK;
}

}  // namespace sde

// Elastic nuclear terms of section 2.1.4 in double precision, shared by the
// host table build (sde_tables.cpp) and the kernels (sde_kernels.hip).
//
// * Elements other than hydrogen: sigma_NI(E) P_NI(mu, E) of Eq.
//   (elastic_large_barns), P_NI a uniform cubic B-spline in mu over [-1, 1]
//   (knot j at -1 + (j - 3) h, h = 2 / m, m = n_mu - 3 intervals).
// * Hydrogen: the nuclear term sigma_N^c(mu, E) of Eq. (hydrogen_not_ruther)
//   for amplitudes a_l (complex) and b_l (real), l < n_l <= 8, and its
//   antiderivative in mu, from the antiderivatives of
//   (1 -+ mu)^-1 cos / sin(eta ln((1 -+ mu) / 2)) (Appendix A.2's
//   recursion) and repeated integration by parts.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace sde {

constexpr int kMaxL = 8;

// P(x) and int_{-1}^{x} P for the spline with coefficients c[0..m+2] over
// [-1, 1]; cum[k] = int_{-1}^{-1 + k h} P (k = 0..m); in the precision R of
// the arrays.
template <class R>
__host__ __device__ inline void ni_spline(const R* c, const R* cum, int m, R x, R& dens,
                                          R& integ) {
    const R h = R(2) / (R)m;
    R t = (x + R(1)) / h;
    t = t < R(0) ? R(0) : (t > (R)m ? (R)m : t);
    int k = (int)t;
    if (k > m - 1) k = m - 1;
    const R u = t - (R)k, v = R(1) - u, u2 = u * u, u3 = u2 * u, u4 = u3 * u;
    const R B0 = v * v * v / R(6), B1 = (R(3) * u3 - R(6) * u2 + R(4)) / R(6),
            B2 = (R(-3) * u3 + R(3) * u2 + R(3) * u + R(1)) / R(6), B3 = u3 / R(6);
    const R I0 = (R(1) - v * v * v * v) / R(24), I1 = (R(0.75) * u4 - R(2) * u3 + R(4) * u) / R(6),
            I2 = (R(-0.75) * u4 + u3 + R(1.5) * u2 + u) / R(6), I3 = u4 / R(24);
    dens = c[k] * B0 + c[k + 1] * B1 + c[k + 2] * B2 + c[k + 3] * B3;
    integ = cum[k] + h * (c[k] * I0 + c[k + 1] * I1 + c[k + 2] * I2 + c[k + 3] * I3);
    if (x <= R(-1)) integ = R(0);
}

// Hydrogen amplitudes at one energy.
struct HAmp {
    int n_l;
    double are[kMaxL], aim[kMaxL], b[kMaxL];
};

// sigma_N^c(mu) (barn/sr) and its antiderivative in mu (barn, up to a
// constant that cancels in every definite integral).
//
// Antiderivative.  The b_l terms integrate through int P_n = (P_{n+1} -
// P_{n-1}) / (2n + 1) (mu for n = 0).  For the a_l terms, Re(a_l e^{i phi}) =
// c1 cos(phi) + c2 sin(phi) with (c1, c2) = (Re a_l, -Im a_l), and with
// y = 1 + sg mu (sg = -1 for the (1 - mu) denominator, +1 for (1 + mu)),
// phi = eta ln(y / 2), the k-th antiderivative of (c1 cos + c2 sin) / y is
// y^(k-1) (cc_k cos + cs_k sin) with cc_0 = c1, cs_0 = c2 and
//   cc_{k+1} = sg (k cc_k - eta cs_k) / (k^2 + eta^2),
//   cs_{k+1} = sg (eta cc_k + k cs_k) / (k^2 + eta^2).
// The recursion is linear in (c1, c2): it runs once for (1, 0) and (0, 1),
// and the monomial moments int mu^n f = sum_{i<=n} (-1)^i n!/(n-i)!
// f^(i+1) mu^(n-i) are combined with each P_l's monomial coefficients.
__host__ __device__ inline void h_nuclear(const HAmp& A, double eta, double mu, double& dens,
                                          double& G) {
    // Legendre values P_0..P_{2 kMaxL} and monomial coefficients of P_0..P_7
    double P[2 * kMaxL + 1];
    P[0] = 1.0;
    P[1] = mu;
    for (int n = 1; n < 2 * kMaxL; ++n) P[n + 1] = ((2.0 * n + 1.0) * mu * P[n] - n * P[n - 1]) / (n + 1.0);
    double mono[kMaxL][kMaxL];   // P_l = sum_n mono[l][n] mu^n
    for (int l = 0; l < kMaxL; ++l)
        for (int n = 0; n < kMaxL; ++n) mono[l][n] = 0.0;
    mono[0][0] = 1.0;
    if (kMaxL > 1) mono[1][1] = 1.0;
    for (int l = 1; l + 1 < kMaxL; ++l)
        for (int n = 0; n < kMaxL; ++n)
            mono[l + 1][n] = ((2.0 * l + 1.0) * (n > 0 ? mono[l][n - 1] : 0.0) -
                              l * mono[l - 1][n]) / (l + 1.0);
    // per denominator: the phase, then the antiderivative moments of the
    // two unit coefficient pairs
    double cosp[2], sinp[2], F[2][2][kMaxL];   // [sign][basis][n]
    for (int sgi = 0; sgi < 2; ++sgi) {
        const double sg = sgi == 0 ? -1.0 : 1.0;
        const double y = 1.0 + sg * mu;
        const double phi = eta * log(0.5 * y);
        cosp[sgi] = cos(phi);
        sinp[sgi] = sin(phi);
        for (int bi = 0; bi < 2; ++bi) {
            double cc = bi == 0 ? 1.0 : 0.0, cs = bi == 0 ? 0.0 : 1.0;
            double fk[kMaxL + 1];   // f^(k), k = 1..kMaxL
            double yp = 1.0;        // y^(k-1)
            for (int k = 0; k < kMaxL; ++k) {
                const double d = k * k + eta * eta;
                const double ncc = sg * (k * cc - eta * cs) / d;
                const double ncs = sg * (eta * cc + k * cs) / d;
                cc = ncc;
                cs = ncs;
                fk[k + 1] = yp * (cc * cosp[sgi] + cs * sinp[sgi]);
                yp *= y;
            }
            for (int n = 0; n < kMaxL; ++n) {
                double s = 0.0, fact = 1.0, mp = 1.0;   // n!/(n-i)!, mu^(n-i) built downward
                double mpow[kMaxL];
                mpow[0] = 1.0;
                for (int q = 1; q <= n; ++q) mpow[q] = mpow[q - 1] * mu;
                for (int i = 0; i <= n; ++i) {
                    if (i > 0) fact *= (n - i + 1);
                    mp = mpow[n - i];
                    s += ((i & 1) ? -fact : fact) * fk[i + 1] * mp;
                }
                F[sgi][bi][n] = s;
            }
        }
    }
    double s1 = 0.0, i1 = 0.0, s2 = 0.0, i2 = 0.0;
    for (int l = 0; l < A.n_l; ++l) {
        const int n2 = 2 * l;
        s1 += (4.0 * l + 1.0) / 2.0 * A.b[l] * P[n2];
        i1 += (4.0 * l + 1.0) / 2.0 * A.b[l] *
              (n2 == 0 ? mu : (P[n2 + 1] - P[n2 - 1]) / (2.0 * n2 + 1.0));
        const double c1 = A.are[l], c2 = -A.aim[l], par = (l & 1) ? -1.0 : 1.0;
        // density: Re{[(1+mu) e^{i phi-} + (-1)^l (1-mu) e^{i phi+}] a_l} P_l
        s2 += (2.0 * l + 1.0) / 2.0 * P[l] *
              ((1.0 + mu) * (c1 * cosp[0] + c2 * sinp[0]) +
               par * (1.0 - mu) * (c1 * cosp[1] + c2 * sinp[1]));
        double acc = 0.0;
        for (int n = 0; n <= l; ++n) {
            const double pn = mono[l][n];
            if (pn == 0.0) continue;
            acc += pn * (c1 * (F[0][0][n] + par * F[1][0][n]) + c2 * (F[0][1][n] + par * F[1][1][n]));
        }
        i2 += (2.0 * l + 1.0) / 2.0 * acc;
    }
    dens = s1 - 2.0 * eta / ((1.0 - mu) * (1.0 + mu)) * s2;
    G = i1 - 2.0 * eta * i2;
}

}  // namespace sde

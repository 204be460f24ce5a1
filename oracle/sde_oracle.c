/*
 * FP64 CPU oracle of the jump-SDE proton transport of Dean, Perez-Lara,
 * Horton, Southerby, Koskela and Kyprianou, "SDE-based Monte Carlo dose
 * calculation for proton therapy validated against Geant4" (arXiv 2511.03115).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity reference for the HIP
 * path: it is plain, slow and written to be checked against the paper by
 * eye.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant
 * generator with the HIP library; the two only read the same seeded inputs.
 *
 * Every physical quantity is evaluated in double precision straight from its
 * defining formula at the state Y_n (explicit Euler-Maruyama).  Where the
 * paper is silent or garbled the reading taken is stated at the function.
 *
 * Units: MeV, cm, g/cm^3, barn (1e-24 cm^2), radians.
 *
 * Parity unpinned (no independent value to compare with): the placeholder
 * nuclear inelastic data.  The small-angle diffusion has two samplers: the
 * spherical Brownian motion law (switch OR_SBM, see sbm_polar; pinned by
 * its heat-kernel moments) and the geodesic Gaussian step (geodesic_step),
 * which approximates it to O(t) in the angle and is pinned by the thin-slab
 * laws only.
 */
#include <complex.h>
#undef I   /* the imaginary unit is written _Complex_I below; I is a variable name */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_ELEM 16
#define OR_MAX_MAT 16
#define OR_RG_LATTICE 4096

/* physics switches */
#define OR_LOSS 1
#define OR_STRAGGLE 2
#define OR_MCS 4
#define OR_ELASTIC 8
#define OR_INELASTIC 16
#define OR_EOR 32
#define OR_SBM 64   /* small-angle diffusion by the spherical Brownian motion law */
#define OR_ECUT 256 /* large-angle elastic cut 2.5 sigma(E) instead of the fixed theta_cut */

/* CODATA 2018 values (the paper does not print them) */
static const double MASS_P = 938.27208816;     /* proton rest energy, MeV */
static const double MASS_E = 0.51099895000;    /* electron rest energy, MeV */
static const double ALPHA = 7.2973525693e-3; /* fine-structure constant */
static const double N_A = 6.02214076e23;    /* 1/mol */
static const double HBARC_FM = 197.3269804; /* MeV fm */
static const double AMU_MEV = 931.49410242; /* MeV per atomic mass unit */
static const double MEV_TO_J = 1.602176634e-13;
/* Bethe-Bloch constant exactly as printed in Eq. (bethbloch) */
static const double BETHE_K = 0.3072;       /* MeV cm^2 / mol */
static const double TWO_PI = 6.283185307179586476925286766559;

typedef struct {
    int n_elem;
    int Z[OR_MAX_ELEM];
    double A[OR_MAX_ELEM];  /* g/mol */
    double w[OR_MAX_ELEM];  /* mass fractions */
    double I_eV;
} or_material;

typedef struct {
    double step_cm;      /* Delta */
    double ld_z_cm;      /* z of the Lynch-Dahl width */
    double e_min;        /* absorption energy */
    double e_max;
    double ld_F;
    double theta_cut;    /* large-angle elastic cut (CM), rad */
    double theta_bs;     /* hydrogen backscatter cut (CM), rad */
    long long max_steps;
    unsigned flags;
    int pad;
} or_params;

typedef struct {
    int n_tab, n_e, n_u, pad;
    double e_lo, e_hi;
    const int* Z;            /* [n_tab] */
    const double* sigma;     /* [n_tab][n_e] barn */
    const double* u_icdf;    /* [n_tab][n_e][n_u] */
    const double* kr;        /* [n_tab][n_e][n_u] */
    const double* ka;        /* [n_tab][n_e][n_u] */
    /* Elastic nuclear data (section 2.1.4).  Elements other than hydrogen:
     * sigma_NI(E_i) in barn and the cubic B-spline coefficients of
     * P_NI(mu, E_i) on uniform knots over [-1, 1] (n_mu >= 4; knot j at
     * -1 + (j - 3) h, h = 2 / (n_mu - 3)).  Hydrogen: partial waves
     * l = 0..n_l-1 (n_l <= 8), the cubic B-spline coefficients in the
     * lattice coordinate (n_e + 2 per l, uniform knots at the lattice
     * points) of Re a_l, Im a_l and b_l (barn). */
    int n_ni, n_mu;
    const int* ni_Z;         /* [n_ni] */
    const double* ni_sigma;  /* [n_ni][n_e] barn */
    const double* ni_p;      /* [n_ni][n_e][n_mu] */
    int n_l, pad2;
    const double* h_are;     /* [n_l][n_e + 2] */
    const double* h_aim;
    const double* h_b;
} or_nuclear;

typedef struct {
    int nx, ny, nz, pad;
    double d[3];
    double origin[3];
    const unsigned char* mat;   /* (nz, ny, nx) */
    const float* rho;           /* (nz, ny, nx) */
} or_phantom;

typedef struct {
    double E, sigmaE, x, y, sigma_xy, weight;
    unsigned long long n;
} or_spot;

/* ------------------------------------------------------------------------ */
/* Philox counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).      */
/* Written once, generic in the word width; the 64-bit instance exists only */
/* so that a test can compare it bit for bit with numpy.random.Philox.      */
/* ------------------------------------------------------------------------ */
#define OR_PHILOX4(NAME, T, WT, M0, M1, W0, W1, BITS)                          \
    void NAME(const T ctr_in[4], const T key_in[2], T out[4]) {                \
        T c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];     \
        T k0 = key_in[0], k1 = key_in[1];                                      \
        for (int r = 0; r < 10; ++r) {                                         \
            if (r > 0) { k0 += (T)(W0); k1 += (T)(W1); }                       \
            WT p0 = (WT)(T)(M0) * (WT)c0;                                      \
            WT p1 = (WT)(T)(M1) * (WT)c2;                                      \
            T hi0 = (T)(p0 >> BITS), lo0 = (T)p0;                              \
            T hi1 = (T)(p1 >> BITS), lo1 = (T)p1;                              \
            T n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;                          \
            c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;                              \
        }                                                                      \
        out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;                    \
    }

OR_PHILOX4(or_philox4x32_10, uint32_t, uint64_t, 0xD2511F53u, 0xCD9E8D57u,
           0x9E3779B9u, 0xBB67AE85u, 32)
OR_PHILOX4(or_philox4x64_10, uint64_t, unsigned __int128, 0xD2E7470EE14C6C93ull,
           0xCA5A826395121157ull, 0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull, 64)

/* Block (h, n, b) of history h, step n, block b, under key = seed. */
static void rng_block(uint64_t seed, uint64_t h, uint32_t n, uint32_t b, uint32_t w[4]) {
    uint32_t ctr[4] = {(uint32_t)h, (uint32_t)(h >> 32), n, b};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, w);
}

/* Uniform on (0,1) from the top 23 bits of a word: (2k+1) 2^-24. */
static double u_hi(uint32_t w) { return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0); }

/* Uniform on (0,1) from the 23 low bits left over by u_hi of w0, w1, w2. */
static double u_lo(uint32_t w0, uint32_t w1, uint32_t w2) {
    uint32_t k = (w0 & 0x1FFu) | ((w1 & 0x1FFu) << 9) | ((w2 & 0x1Fu) << 18);
    return ((double)k + 0.5) * (1.0 / 8388608.0);
}

/* Exported for the RNG tests. */
void or_rng_block(uint64_t seed, uint64_t h, uint32_t n, uint32_t b, uint32_t* w) {
    rng_block(seed, h, n, b, w);
}
void or_rng_blocks(uint64_t seed, size_t count, const uint64_t* h, const uint32_t* n,
                   const uint32_t* b, uint32_t* w) {
    for (size_t i = 0; i < count; ++i) rng_block(seed, h[i], n[i], b[i], w + 4 * i);
}

/* ------------------------------------------------------------------------ */
/* Kinematics                                                               */
/* ------------------------------------------------------------------------ */

/* beta^2 of a proton of kinetic energy E (section 2.1, below Eq. (bethbloch)). */
static double beta2_of(double E) {
    double g = MASS_P + E;
    return (2.0 * MASS_P + E) * E / (g * g);
}

/* Sum_i w_i Z_i / A_i (mol/g), the Bragg-additivity weight. */
static double zoa(const or_material* m) {
    double s = 0.0;
    for (int i = 0; i < m->n_elem; ++i) s += m->w[i] * m->Z[i] / m->A[i];
    return s;
}

/* Mass stopping power S/rho in MeV cm^2/g: Eq. (bethbloch) with Bragg
 * additivity, Eq. (BraggAditivty), one mean excitation energy per material,
 * no shell, density, Lindhard-Sorensen or Barkas corrections. */
static double stopping_mass(const or_material* m, double E) {
    double b2 = beta2_of(E);
    double I = m->I_eV * 1e-6;
    double L = log(2.0 * MASS_E * b2 / (I * (1.0 - b2))) - b2;
    return BETHE_K * zoa(m) / b2 * L;
}

/* Straggling variance per unit length and density, MeV^2 cm^2/g:
 * Eq. (energystraggling) with Bragg additivity. */
static double straggle_mass(const or_material* m, double E) {
    double b2 = beta2_of(E);
    double g = 1.0 + E / MASS_P;
    double ahc_cm = ALPHA * HBARC_FM * 1e-13;   /* alpha hbar c in MeV cm */
    return 4.0 * M_PI * N_A * zoa(m) * ahc_cm * ahc_cm * g * g * (1.0 - 0.5 * b2);
}

/* Lynch-Dahl Gaussian width sigma(E) after path z (section 2.1,
 * "Moliere's theory for small-angle elastic scattering"), with the square
 * root the paper restores.  Compound: chi_c^2 summed over elements with
 * thickness rho w_i z; ln chi_alpha^2 averaged with weights
 * w_i Z_i (Z_i + 1) / A_i (the mass fraction enters as in Lynch and Dahl,
 * since each element's chi_c^2 carries its own thickness). */
static double lynch_dahl_sigma(const or_material* m, double rho, double E, double z, double F) {
    double p2 = E * E + 2.0 * E * MASS_P;
    double pbeta = p2 / (E + MASS_P);
    double b2 = beta2_of(E);
    double chic2 = 0.0, num = 0.0, den = 0.0;
    for (int i = 0; i < m->n_elem; ++i) {
        double Z = m->Z[i];
        double wz = m->w[i] * Z * (Z + 1.0) / m->A[i];
        chic2 += 0.157 * wz * rho * z / (pbeta * pbeta);
        double za = Z * ALPHA;
        double chia2 = 2.007e-5 * pow(Z, 2.0 / 3.0) * (1.0 + 3.34 * za * za / b2) / p2;
        num += wz * log(chia2);
        den += wz;
    }
    double chia2 = exp(num / den);
    double nu = chic2 / (2.0 * chia2 * (1.0 - F));
    double s2 = chic2 / (1.0 + F * F) * ((1.0 + nu) / nu * log1p(nu) - 1.0);
    return sqrt(s2);
}

/* (eta/k)^2 in fm^2 for a proton on a nucleus (Z, A): section 2.1,
 * "Large angle elastic scattering", with eta = Z alpha sqrt(m_p/(2E)) and
 * k = A/(1+A) sqrt(2 m_p E)/(hbar c); the printed 1e-26 and 1e6 unit
 * factors are read as garbled and dropped. */
static double eta2_over_k2_fm2(double Z, double A, double E) {
    double ahc = ALPHA * HBARC_FM;
    double r = Z * ahc * (1.0 + A) / (2.0 * A * E);
    return r * r;
}

/* 1 - cos(t) without cancellation. */
static double one_minus_cos(double t) { double s = sin(0.5 * t); return 2.0 * s * s; }

/* Integral over mu in [-1, cos(theta_cut)] of the unscreened CM Rutherford
 * cross section sigma_R = (eta/k)^2 / (1-mu)^2, in barn (Eq. (large_elastic_cm)
 * with sigma_NI = 0). */
static double rutherford_integral_barn(double Z, double A, double E, double theta_cut) {
    double T = 1.0 / one_minus_cos(theta_cut);
    return eta2_over_k2_fm2(Z, A, E) * (T - 0.5) * 0.01;
}

/* Mott (identical-particle Rutherford) antiderivative for hydrogen,
 * Appendix A.2, in units of (eta/k)^2 barn:
 *   G(mu) = 2 mu/(1-mu^2) - sin(eta ln((1+mu)/(1-mu))) / (2 eta).
 * The printed form has sin(2 eta ln ...); its derivative does not give the
 * Mott cross section of section 2.1, the form above does, so it is used. */
static double mott_G(double eta, double mu) {
    return 2.0 * mu / (1.0 - mu * mu) - sin(eta * log((1.0 + mu) / (1.0 - mu))) / (2.0 * eta);
}

static double mott_eta(double E) { return ALPHA * sqrt(MASS_P / (2.0 * E)); }

/* Integral of the Mott cross section over [-cos(theta_bs), cos(theta_cut)],
 * Eq. (large_elastic_cm_hydrogen) with sigma_N = 0, in barn. */
static double mott_integral_barn(double A, double E, double theta_cut, double theta_bs) {
    double eta = mott_eta(E);
    double hi = cos(theta_cut), lo = -cos(theta_bs);
    return eta2_over_k2_fm2(1.0, A, E) * (mott_G(eta, hi) - mott_G(eta, lo)) * 0.01;
}

/* Position of E on the nuclear-table lattice (uniform in ln E). */
static void lattice_pos(const or_nuclear* nu, double E, int* i, double* f) {
    double t = (log(E) - log(nu->e_lo)) / (log(nu->e_hi) - log(nu->e_lo)) * (nu->n_e - 1);
    if (t < 0.0) t = 0.0;
    if (t > nu->n_e - 1) t = nu->n_e - 1;
    int k = (int)floor(t);
    if (k > nu->n_e - 2) k = nu->n_e - 2;
    *i = k;
    *f = t - k;
}

static int nuclear_row(const or_nuclear* nu, int Z) {
    if (!nu) return -1;
    for (int t = 0; t < nu->n_tab; ++t) if (nu->Z[t] == Z) return t;
    return -1;
}

/* Inelastic cross section in barn, linear between lattice points
 * (section 2.1, "Parameterisation for inelastic proton-nucleus
 * interactions"; the paper's cubic B-spline fit needs the ENDF data). */
static double inelastic_sigma_barn(const or_nuclear* nu, int t, double E) {
    int i; double f;
    lattice_pos(nu, E, &i, &f);
    const double* s = nu->sigma + (size_t)t * nu->n_e;
    return (1.0 - f) * s[i] + f * s[i + 1];
}

/* Bilinear interpolation of a [n_e][n_u] table at (E, x in [0,1]). */
static double table_eu(const or_nuclear* nu, const double* tab, double E, double x) {
    int i; double f;
    lattice_pos(nu, E, &i, &f);
    double tu = x * (nu->n_u - 1);
    if (tu < 0.0) tu = 0.0;
    if (tu > nu->n_u - 1) tu = nu->n_u - 1;
    int j = (int)floor(tu);
    if (j > nu->n_u - 2) j = nu->n_u - 2;
    double g = tu - j;
    const double* r0 = tab + (size_t)i * nu->n_u;
    const double* r1 = tab + (size_t)(i + 1) * nu->n_u;
    double a = (1.0 - g) * r0[j] + g * r0[j + 1];
    double b = (1.0 - g) * r1[j] + g * r1[j + 1];
    return (1.0 - f) * a + f * b;
}

/* ------------------------------------------------------------------------ */
/* Elastic nuclear terms (section 2.1.4)                                    */
/* ------------------------------------------------------------------------ */

/* The uniform cubic B-spline basis on one knot interval, at local u in [0, 1]:
 * the four pieces (1-u)^3/6, (3u^3 - 6u^2 + 4)/6, (-3u^3 + 3u^2 + 3u + 1)/6,
 * u^3/6 of the cardinal cubic B-spline. */
static void bspline3_basis(double u, double B[4]) {
    double v = 1.0 - u;
    B[0] = v * v * v / 6.0;
    B[1] = (3.0 * u * u * u - 6.0 * u * u + 4.0) / 6.0;
    B[2] = (-3.0 * u * u * u + 3.0 * u * u + 3.0 * u + 1.0) / 6.0;
    B[3] = u * u * u / 6.0;
}

/* Value at x of the cubic spline with coefficients c[0..m+2] on the uniform
 * knots x0 + (j - 3) h (m intervals covering [x0, x0 + m h]); x is clamped
 * to that range. */
static double bspline3(const double* c, int m, double x0, double h, double x) {
    double t = (x - x0) / h;
    if (t < 0.0) t = 0.0;
    if (t > m) t = m;
    int k = (int)floor(t);
    if (k > m - 1) k = m - 1;
    double B[4];
    bspline3_basis(t - k, B);
    return c[k] * B[0] + c[k + 1] * B[1] + c[k + 2] * B[2] + c[k + 3] * B[3];
}

/* P_NI of element row t at lattice energy i and cosine mu. */
static double p_ni(const or_nuclear* nu, int t, int i, double mu) {
    int m = nu->n_mu - 3;
    const double* c = nu->ni_p + ((size_t)t * nu->n_e + i) * nu->n_mu;
    return bspline3(c, m, -1.0, 2.0 / m, mu);
}

/* int_{-1}^{x} P_NI(mu, E_i) dmu: 4-point Gauss-Legendre on every knot
 * interval (exact for the cubic pieces). */
static double p_ni_integral(const or_nuclear* nu, int t, int i, double x) {
    static const double gx[4] = {-0.86113631159405257522, -0.33998104358485626480,
                                 0.33998104358485626480, 0.86113631159405257522};
    static const double gw[4] = {0.34785484513745385737, 0.65214515486254614263,
                                 0.65214515486254614263, 0.34785484513745385737};
    int m = nu->n_mu - 3;
    double h = 2.0 / m, s = 0.0;
    if (x <= -1.0) return 0.0;
    if (x > 1.0) x = 1.0;
    for (int k = 0; k < m; ++k) {
        double a = -1.0 + k * h, b = a + h;
        if (a >= x) break;
        if (b > x) b = x;
        double c = 0.5 * (a + b), r = 0.5 * (b - a);
        for (int q = 0; q < 4; ++q) s += gw[q] * r * p_ni(nu, t, i, c + r * gx[q]);
    }
    return s;
}

static int ni_row(const or_nuclear* nu, int Z) {
    if (!nu || nu->n_ni <= 0) return -1;
    for (int t = 0; t < nu->n_ni; ++t) if (nu->ni_Z[t] == Z) return t;
    return -1;
}

/* The nuclear-plus-interference term sigma_NI(E) P_NI(mu, E) of Eq.
 * (elastic_large_barns) at energy E, linear in the lattice coordinate
 * between the two neighbouring lattice energies (the paper extends its
 * lattice quantities linearly): its density in mu (barn/sr) and its
 * integral from -1 to x (barn). */
static double ni_density(const or_nuclear* nu, int t, double E, double mu) {
    int i; double f;
    lattice_pos(nu, E, &i, &f);
    const double* sg = nu->ni_sigma + (size_t)t * nu->n_e;
    return (1.0 - f) * sg[i] * p_ni(nu, t, i, mu) + f * sg[i + 1] * p_ni(nu, t, i + 1, mu);
}
static double ni_integral(const or_nuclear* nu, int t, double E, double x) {
    int i; double f;
    lattice_pos(nu, E, &i, &f);
    const double* sg = nu->ni_sigma + (size_t)t * nu->n_e;
    return (1.0 - f) * sg[i] * p_ni_integral(nu, t, i, x) +
           f * sg[i + 1] * p_ni_integral(nu, t, i + 1, x);
}

/* Hydrogen partial-wave amplitudes at E: the cubic B-splines in the lattice
 * coordinate (section 2.1.4: a_l(E), b_l(E) extended by a cubic B-spline). */
static void h_amplitudes(const or_nuclear* nu, double E, double complex* a, double* b) {
    double t = (log(E) - log(nu->e_lo)) / (log(nu->e_hi) - log(nu->e_lo)) * (nu->n_e - 1);
    int m = nu->n_e - 1;
    for (int l = 0; l < nu->n_l; ++l) {
        const double* cr = nu->h_are + (size_t)l * (nu->n_e + 2);
        const double* ci = nu->h_aim + (size_t)l * (nu->n_e + 2);
        const double* cb = nu->h_b + (size_t)l * (nu->n_e + 2);
        a[l] = bspline3(cr, m, 0.0, 1.0, t) + _Complex_I * bspline3(ci, m, 0.0, 1.0, t);
        b[l] = bspline3(cb, m, 0.0, 1.0, t);
    }
}

/* Legendre polynomial P_n(x) by the three-term recurrence. */
static double legendre(int n, double x) {
    double pm = 1.0, p = x;
    if (n == 0) return 1.0;
    for (int k = 1; k < n; ++k) {
        double pn = ((2.0 * k + 1.0) * x * p - k * pm) / (k + 1.0);
        pm = p;
        p = pn;
    }
    return p;
}

/* The hydrogen nuclear term sigma_N^c(mu, E) of Eq. (hydrogen_not_ruther),
 * barn/sr, evaluated literally (eta = alpha sqrt(m_p / 2E)). */
static double h_nuclear_density(const or_nuclear* nu, double E, double mu) {
    double complex a[8];
    double b[8];
    h_amplitudes(nu, E, a, b);
    double eta = mott_eta(E);
    double s1 = 0.0;
    double complex s2 = 0.0;
    double complex em = cexp(_Complex_I * eta * log((1.0 - mu) / 2.0));
    double complex ep = cexp(_Complex_I * eta * log((1.0 + mu) / 2.0));
    for (int l = 0; l < nu->n_l; ++l) {
        s1 += (4.0 * l + 1.0) / 2.0 * b[l] * legendre(2 * l, mu);
        double sgn = (l % 2) ? -1.0 : 1.0;
        s2 += ((1.0 + mu) * em + sgn * (1.0 - mu) * ep) * (2.0 * l + 1.0) / 2.0 * a[l] *
              legendre(l, mu);
    }
    return s1 - 2.0 * eta / (1.0 - mu * mu) * creal(s2);
}

/* Coefficients of P_l(x) = sum_n p[n] x^n, l <= 15, by the recurrence on
 * coefficient vectors. */
static void legendre_monomials(int l, double* p) {
    double pm[16] = {0}, pc[16] = {0}, pn[16];
    pm[0] = 1.0;          /* P_0 */
    pc[1] = 1.0;          /* P_1 */
    if (l == 0) { memcpy(p, pm, sizeof pm); return; }
    for (int k = 1; k < l; ++k) {
        for (int n = 0; n < 16; ++n) {
            double up = n > 0 ? pc[n - 1] : 0.0;
            pn[n] = ((2.0 * k + 1.0) * up - k * pm[n]) / (k + 1.0);
        }
        memcpy(pm, pc, sizeof pc);
        memcpy(pc, pn, sizeof pn);
    }
    memcpy(p, pc, sizeof pc);
}

/* Antiderivative (Appendix A.2) of mu^n f(mu), f(mu) = (c1 cos(phi) +
 * c2 sin(phi)) / (1 + sg mu), phi = eta ln((1 + sg mu) / 2), sg = +1 or -1:
 * the k-th antiderivative of f is (1 + sg mu)^(k-1) (cc_k cos(phi) +
 * cs_k sin(phi)) with cc_0 = c1, cs_0 = c2 and
 *   cc_{k+1} = sg (k cc_k - eta cs_k) / (k^2 + eta^2),
 *   cs_{k+1} = sg (eta cc_k + k cs_k) / (k^2 + eta^2),
 * and by repeated integration by parts
 *   int mu^n f = sum_{i=0}^{n} (-1)^i n! / (n-i)! f^(i+1)(mu) mu^(n-i)
 * up to a constant (it cancels in every definite integral taken here). */
static double h_mono_antiderivative(int n, double sg, double c1, double c2, double eta,
                                    double mu) {
    double cc[17], cs[17];
    cc[0] = c1;
    cs[0] = c2;
    for (int k = 0; k <= n; ++k) {
        double d = k * k + eta * eta;
        cc[k + 1] = sg * (k * cc[k] - eta * cs[k]) / d;
        cs[k + 1] = sg * (eta * cc[k] + k * cs[k]) / d;
    }
    double y = 1.0 + sg * mu;
    double phi = eta * log(y / 2.0), cp = cos(phi), sp = sin(phi);
    double s = 0.0, fact = 1.0;   /* n! / (n - i)! */
    for (int i = 0; i <= n; ++i) {
        if (i > 0) fact *= (n - i + 1);
        double fi = pow(y, i) * (cc[i + 1] * cp + cs[i + 1] * sp);   /* f^(i+1) */
        s += ((i % 2) ? -1.0 : 1.0) * fact * fi * pow(mu, n - i);
    }
    return s;
}

/* Antiderivative in mu of sigma_N^c(mu, E) (barn): the b_l terms through
 * int P_n = (P_{n+1} - P_{n-1}) / (2n + 1) (x for n = 0), the a_l terms
 * through h_mono_antiderivative with c1 = Re a_l, c2 = -Im a_l (so that
 * c1 cos + c2 sin = Re(a_l e^{i phi})) for the (1 - mu) and (1 + mu)
 * denominators. */
static double h_nuclear_antiderivative(const or_nuclear* nu, double E, double mu) {
    double complex a[8];
    double b[8];
    h_amplitudes(nu, E, a, b);
    double eta = mott_eta(E);
    double s1 = 0.0, s2 = 0.0;
    for (int l = 0; l < nu->n_l; ++l) {
        int n2 = 2 * l;
        double ip = n2 == 0 ? mu : (legendre(n2 + 1, mu) - legendre(n2 - 1, mu)) / (2.0 * n2 + 1.0);
        s1 += (4.0 * l + 1.0) / 2.0 * b[l] * ip;
        double p[16];
        legendre_monomials(l, p);
        double c1 = creal(a[l]), c2 = -cimag(a[l]), sgn = (l % 2) ? -1.0 : 1.0;
        double acc = 0.0;
        for (int n = 0; n <= l; ++n) {
            if (p[n] == 0.0) continue;
            acc += p[n] * (h_mono_antiderivative(n, -1.0, c1, c2, eta, mu) +
                           sgn * h_mono_antiderivative(n, +1.0, c1, c2, eta, mu));
        }
        s2 += (2.0 * l + 1.0) / 2.0 * acc;
    }
    return s1 - 2.0 * eta * s2;
}

/* ------------------------------------------------------------------------ */
/* Jump channels (Eq. (Npi)): for compounds each element is an independent  */
/* point process (section 2.1), elastic and inelastic per element.          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    double theta_c;                /* the elastic cut (CM), rad */
    double rate[2 * OR_MAX_ELEM];  /* per cm */
    int elem[2 * OR_MAX_ELEM];
    int inel[2 * OR_MAX_ELEM];
    int tab[2 * OR_MAX_ELEM];
} channels;

/* The large-angle elastic cut at E in medium m of density rho.  Fixed:
 * theta_cut, as the paper's runs take it.  With OR_ECUT: 2.5 sigma(E), sigma
 * the Lynch-Dahl width of section 2.1.4 for this medium and density over the
 * path z of that width (the cut the paper states and names as energy
 * dependent), applied to the CM angle like the fixed cut. */
static double elastic_cut(const or_material* m, const or_params* p, double rho, double E) {
    if (!(p->flags & OR_ECUT)) return p->theta_cut;
    return 2.5 * lynch_dahl_sigma(m, rho, E, p->ld_z_cm, p->ld_F);
}

/* The cut limited to the range where the law is defined: pi for Rutherford
 * (the rate vanishes there), pi - theta_bs for hydrogen (the interval
 * [-cos theta_bs, cos theta_c] closes there). */
static double cut_for(int Z, double theta_c, double theta_bs) {
    double top = (Z == 1) ? M_PI - theta_bs : M_PI;
    return theta_c < top ? theta_c : top;
}

/* The elastic nuclear terms' integral (barn) over the CM cosines of the
 * large-angle law: sigma_NI P_NI from -1 to cos(cut) for elements with
 * such data, sigma_N from -cos(theta_bs) to cos(cut) for hydrogen with
 * partial waves; 0 without data. */
static double elastic_nuclear_integral_barn(const or_nuclear* nu, int Z, double E, double tc,
                                            double theta_bs) {
    if (!nu) return 0.0;
    if (Z == 1) {
        if (nu->n_l <= 0) return 0.0;
        double hi = cos(tc), lo = -cos(theta_bs);
        if (hi <= lo) return 0.0;
        return h_nuclear_antiderivative(nu, E, hi) - h_nuclear_antiderivative(nu, E, lo);
    }
    int t = ni_row(nu, Z);
    return t < 0 ? 0.0 : ni_integral(nu, t, E, cos(tc));
}

static void channel_rates(const or_material* m, const or_nuclear* nu, const or_params* p,
                          double rho, double E, channels* c) {
    c->n = 0;
    c->theta_c = elastic_cut(m, p, rho, E);
    for (int i = 0; i < m->n_elem; ++i) {
        double nd = N_A * rho * m->w[i] / m->A[i];    /* atoms per cm^3 */
        if (p->flags & OR_ELASTIC) {
            double tc = cut_for(m->Z[i], c->theta_c, p->theta_bs);
            double xs = (m->Z[i] == 1)
                ? mott_integral_barn(m->A[i], E, tc, p->theta_bs)
                : rutherford_integral_barn(m->Z[i], m->A[i], E, tc);
            xs += elastic_nuclear_integral_barn(nu, m->Z[i], E, tc, p->theta_bs);
            /* 2 pi from the azimuth, 1e-24 cm^2 per barn (Eq. (large_elastic_cm)) */
            c->rate[c->n] = 2.0 * M_PI * nd * xs * 1e-24;
            c->elem[c->n] = i; c->inel[c->n] = 0; c->tab[c->n] = -1;
            c->n++;
        }
        if (p->flags & OR_INELASTIC) {
            int t = nuclear_row(nu, m->Z[i]);
            if (t >= 0) {
                c->rate[c->n] = nd * inelastic_sigma_barn(nu, t, E) * 1e-24;
                c->elem[c->n] = i; c->inel[c->n] = 1; c->tab[c->n] = t;
                c->n++;
            }
        }
    }
}

/* Sample the CM cosine of a non-hydrogen elastic jump by inverting the
 * closed-form Rutherford CDF, Eq. (large_elastic_cdf) with sigma_NI = 0:
 *   Pi(nu) = (1/(1-nu) - 1/2) / (1/(1-mu_c) - 1/2).
 * Returns 1 - mu, which keeps the forward angles accurate. */
static double rutherford_one_minus_mu(double U, double theta_cut) {
    double T = 1.0 / one_minus_cos(theta_cut);
    return 1.0 / (0.5 + U * (T - 0.5));
}

/* Sample the CM cosine of a hydrogen elastic jump: solve
 * (G(mu) - G(lo)) / (G(hi) - G(lo)) = U by bisection on the exact Mott
 * antiderivative (the CDF of Eq. (large_elastic_cdf) for hydrogen). */
static double mott_sample_mu(double E, double U, double theta_cut, double theta_bs) {
    double eta = mott_eta(E);
    double lo = -cos(theta_bs), hi = cos(theta_cut);
    double G0 = mott_G(eta, lo), G1 = mott_G(eta, hi);
    double target = G0 + U * (G1 - G0);
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (a + b);
        if (mid <= a || mid >= b) break;
        if (mott_G(eta, mid) < target) a = mid; else b = mid;
    }
    return 0.5 * (a + b);
}

/* The CM cosine of an elastic jump with nuclear data: solve
 * Pi_e(E; nu) = U for the distribution function Eq. (large_elastic_cdf) of
 * the summed cross section (Coulomb + nuclear) by bisection, the numerator
 * the integral from the lower limit (-1, or -cos(theta_bs) for hydrogen). */
static double elastic_cum_barn(const or_nuclear* nu, int Z, double A, double E, double lo,
                               double x) {
    if (Z == 1) {
        double ek2 = eta2_over_k2_fm2(1.0, A, E) * 0.01, eta = mott_eta(E);
        double s = ek2 * (mott_G(eta, x) - mott_G(eta, lo));
        if (nu && nu->n_l > 0)
            s += h_nuclear_antiderivative(nu, E, x) - h_nuclear_antiderivative(nu, E, lo);
        return s;
    }
    double ek2 = eta2_over_k2_fm2(Z, A, E) * 0.01;
    double s = ek2 * (1.0 / (1.0 - x) - 0.5);   /* int_{-1}^{x} (eta/k)^2 / (1 - mu)^2 */
    int t = ni_row(nu, Z);
    if (t >= 0) s += ni_integral(nu, t, E, x);
    return s;
}
static double elastic_sample_mu(const or_nuclear* nu, int Z, double A, double E, double U,
                                double tc, double theta_bs) {
    double lo = (Z == 1) ? -cos(theta_bs) : -1.0, hi = cos(tc);
    double target = U * elastic_cum_barn(nu, Z, A, E, lo, hi);
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (a + b);
        if (mid <= a || mid >= b) break;
        if (elastic_cum_barn(nu, Z, A, E, lo, mid) < target) a = mid; else b = mid;
    }
    return 0.5 * (a + b);
}

/* Kalbach-Mann CM cosine (section 2.1, inelastic): inverse of the CDF of
 * a/(2 sinh a) (cosh(a mu) + r sinh(a mu)).  The printed inverse is
 * exp(a mu); the cosine is its logarithm over a:
 *   mu = ln[(C + sqrt(C^2 - r^2 + 1)) / (1 + r)] / a,
 *   C  = 2 sinh(a) U + r cosh(a) - sinh(a). */
static double kalbach_mu(double a, double r, double U) {
    if (a < 1e-6) return 2.0 * U - 1.0;
    double C = 2.0 * sinh(a) * U + r * cosh(a) - sinh(a);
    double mu = log((C + sqrt(C * C - r * r + 1.0)) / (1.0 + r)) / a;
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    return mu;
}

/* Inelastic event of element table t at E (section 2.1, inelastic
 * proton-nucleus interactions): the loss fraction u from the pi_ne inverse
 * CDF at U1 (linear in E on the lattice and in U), then the CM cosine from
 * the Kalbach-Mann law with r(E, u) and a(E, u) at U3. */
static void inelastic_draw(const or_nuclear* nu, int t, double E, double U1, double U3,
                           double* u_loss, double* cos_cm) {
    size_t off = (size_t)t * nu->n_e * nu->n_u;
    double u = table_eu(nu, nu->u_icdf + off, E, U1);
    if (u < 0.0) u = 0.0;
    if (u > 1.0) u = 1.0;
    double a = table_eu(nu, nu->ka + off, E, u);
    double r = table_eu(nu, nu->kr + off, E, u);
    *u_loss = u;
    *cos_cm = kalbach_mu(a, r, U3);
}

/* CM -> lab polar angle, Appendix A.1, Eq. (cm_to_lab):
 *   tan(theta_L) = sin(theta_CM) / (gamma_u (cos(theta_CM) + u / v'_1C)),
 * taken with atan2.  m1 = m_p, m2 = A amu, K = E_n, outgoing lab energy
 * E_1L - E* with E* = u_loss E_n (zero for elastic). */
static double cm_to_lab(double K, double A, double cos_cm, double sin_cm, double u_loss) {
    double m1 = MASS_P, m2 = A * AMU_MEV;
    double E1 = K + m1;
    double p1 = sqrt(E1 * E1 - m1 * m1);
    double u = p1 / (E1 + m2);
    double gu = 1.0 / sqrt(1.0 - u * u);
    double E1p = E1 - u_loss * K;
    double p1p = sqrt(fmax(E1p * E1p - m1 * m1, 0.0));
    double v1c = (p1p - u * E1p) / (E1p - u * p1p);
    return atan2(sin_cm, gu * (cos_cm + u / v1c));
}

/* ------------------------------------------------------------------------ */
/* Direction updates on S^2                                                  */
/* ------------------------------------------------------------------------ */

/* Orthonormal basis of the plane normal to unit n, branch-free form of
 * Duff, Burgess, Christensen, Hery, Kensler, Liani and Villemin, "Building
 * an Orthonormal Basis, Revisited" (JCGT 6(1), 2017). */
static void onb(const double n[3], double b1[3], double b2[3]) {
    double sign = copysign(1.0, n[2]);
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    b1[0] = 1.0 + sign * n[0] * n[0] * a; b1[1] = sign * b; b1[2] = -sign * n[0];
    b2[0] = b; b2[1] = sign + n[1] * n[1] * a; b2[2] = -n[1];
}

/* Turn d by polar angle theta (given as cos, sin) about itself, azimuth phi
 * measured from b1 of onb(d). */
static void turn(double d[3], double ct, double st, double phi) {
    double b1[3], b2[3], r[3];
    onb(d, b1, b2);
    double cp = cos(phi), sp = sin(phi);
    for (int k = 0; k < 3; ++k) r[k] = ct * d[k] + st * (cp * b1[k] + sp * b2[k]);
    d[0] = r[0]; d[1] = r[1]; d[2] = r[2];
}

/* Aggregated small-angle scattering over one step (section 2.2.2): the
 * time-Delta increment of spherical Brownian motion with volatility
 * m = sigma(E)/sqrt(z), i.e. run for time t = m^2 Delta = sigma^2 Delta/z
 * under the generator (1/2) Laplace-Beltrami on S^2, so that for small t the
 * tangent displacement has per-axis variance t.
 *
 * Geodesic (exponential-map) Gaussian step: polar angle sqrt(t) sqrt(-2 ln U1)
 * (Rayleigh), uniform azimuth 2 pi U2.  Its law differs from the spherical
 * Brownian motion at O(t) in the angle (E[cos] = 1 - t + t^2/3 - ... against
 * e^{-t}). */
static void geodesic_step(double d[3], double sigma_step, double U1, double U2) {
    double th = sigma_step * sqrt(-2.0 * log(U1));
    turn(d, cos(th), sin(th), TWO_PI * U2);
}

/* Spherical Brownian motion on S^2 (d = 3) at time t from the north pole,
 * the sampler the paper cites (Mijatovic, Mramor and Uribe Bravo 2020,
 * Algorithm 1), in two regimes split at SBM_T_SWITCH.
 *
 * Algorithm 1: M = A(t), the number of lineages left at time t of Kingman's
 * coalescent with mutation parameter theta = d - 1 = 2 started from
 * infinitely many (each of k lineages is lost at rate k (k + theta - 1) / 2);
 * X ~ Beta((d-1)/2, (d-1)/2 + M) = Beta(1, 1 + M); cos(angle) = 1 - 2 X,
 * azimuth uniform.  For small t the count M is drawn from Griffiths' (1984)
 * normal law with mean sbm_lineage_mean(t) and variance sbm_lineage_var(t),
 * rounded to the nearest integer and floored at 0, which is how the cited
 * method treats small t: its exact series for P(A(t) = m) cancels
 * catastrophically there (terms ~1e11 at t = 0.05 for values ~0.1).
 *
 * For t >= SBM_T_SWITCH, where that series is still out of reach in double
 * precision but the heat kernel's Legendre series converges within
 * SBM_LEGENDRE_L terms, cos(angle) is drawn exactly by inverting the
 * distribution function of that series (sbm_upper_tail) by bisection.
 *
 * Random inputs: z a standard normal (the lineage count, small t only), u a
 * uniform on (0, 1), oriented so that u -> 1 gives the angle -> 0 in both
 * regimes.  The azimuth is the caller's. */
/* The regime switch is the implementation's choice (the paper cites the
 * sampler, not a switch); the decision is taken on t in double precision. */
#define SBM_T_SWITCH 0.02
#define SBM_LEGENDRE_L 64

/* Griffiths' mean of A(t): 2 eta / t with beta = (theta - 1) t / 2 = t / 2 and
 * eta = beta / (e^beta - 1), i.e. 1 / expm1(t / 2). */
static double sbm_lineage_mean(double t) { return 1.0 / expm1(0.5 * t); }

/* Griffiths' variance of A(t): (2 eta / t) (eta + beta)^2
 * (1 + eta / (eta + beta) - 2 eta) / beta^2.  The bracket is ~beta^2 / 3 and
 * cancels in double precision for small t, so below t = 1e-2 its Taylor
 * series (derived from the same expression) is used: 2 / (3 t) times
 * (1 - 7 t^2 / 240 + 41 t^4 / 80640), truncation O(t^6). */
static double sbm_lineage_var(double t) {
    if (t < 1e-2) {
        double t2 = t * t;
        return 2.0 / (3.0 * t) * (1.0 - 7.0 * t2 / 240.0 + 41.0 * t2 * t2 / 80640.0);
    }
    double beta = 0.5 * t, eta = beta / expm1(beta);
    return (2.0 * eta / t) * (eta + beta) * (eta + beta) *
           (1.0 + eta / (eta + beta) - 2.0 * eta) / (beta * beta);
}

/* P(cos(angle) > c) for spherical Brownian motion at time t: the heat kernel
 * on S^2 is sum_l (2l+1)/2 e^{-l(l+1)t/2} P_l(c) in c, and the integral of
 * P_l from c to 1 is (P_{l-1}(c) - P_{l+1}(c)) / (2l+1) for l >= 1. */
static double sbm_upper_tail(double t, double c) {
    double g = 0.5 * (1.0 - c);
    double pm = 1.0, p = c;                  /* P_{l-1}, P_l at l = 1 */
    for (int l = 1; l <= SBM_LEGENDRE_L; ++l) {
        double pn = ((2.0 * l + 1.0) * c * p - l * pm) / (l + 1.0);   /* P_{l+1} */
        g += 0.5 * exp(-0.5 * l * (l + 1.0) * t) * (pm - pn);
        pm = p;
        p = pn;
    }
    return g;
}

static void sbm_polar(double t, double z, double u, double* ct, double* st) {
    if (t <= 0.0) { *ct = 1.0; *st = 0.0; return; }    /* no motion */
    if (t < SBM_T_SWITCH) {
        double M = floor(sbm_lineage_mean(t) + sqrt(sbm_lineage_var(t)) * z + 0.5);
        if (M < 0.0) M = 0.0;
        double X = -expm1(log(u) / (1.0 + M));          /* Beta(1, 1 + M) by inversion */
        *ct = 1.0 - 2.0 * X;
        *st = 2.0 * sqrt(X * (1.0 - X));
        return;
    }
    /* P(cos(angle) <= c) = u, i.e. sbm_upper_tail(t, c) = 1 - u */
    double lo = -1.0, hi = 1.0;
    for (int i = 0; i < 60; ++i) {
        double c = 0.5 * (lo + hi);
        if (sbm_upper_tail(t, c) > 1.0 - u) lo = c; else hi = c;
    }
    double c = 0.5 * (lo + hi);
    *ct = c;
    *st = sqrt((1.0 - c) * (1.0 + c));
}

static void normalize(double d[3]) {
    double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    d[0] /= n; d[1] /= n; d[2] /= n;
}

/* ------------------------------------------------------------------------ */
/* Residual range (end of range): R_g(E) = int_{e_min}^{E} dE' / (S/rho).   */
/* ------------------------------------------------------------------------ */
static double gl_x[16], gl_w[16];
static int gl_ready = 0;

/* 16-point Gauss-Legendre nodes by Newton iteration on P_16. */
static void gl_init(void) {
    if (gl_ready) return;
    const int n = 16;
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = pk;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        gl_x[i] = x;
        gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    gl_ready = 1;
}

static double range_panel(const or_material* m, double a, double b) {
    double c = 0.5 * (a + b), h = 0.5 * (b - a), s = 0.0;
    for (int i = 0; i < 16; ++i) s += gl_w[i] / stopping_mass(m, c + h * gl_x[i]);
    return s * h;
}

typedef struct {
    double lnlo, dln;
    double E[OR_RG_LATTICE];
    double Rg[OR_RG_LATTICE];   /* exact cumulative at E[j] */
} range_cache;

static void range_cache_init(const or_material* m, double e_min, double e_max, range_cache* rc) {
    rc->lnlo = log(e_min);
    rc->dln = (log(e_max) - log(e_min)) / (OR_RG_LATTICE - 1);
    rc->E[0] = e_min;
    rc->Rg[0] = 0.0;
    for (int j = 1; j < OR_RG_LATTICE; ++j) {
        rc->E[j] = exp(rc->lnlo + j * rc->dln);
        rc->Rg[j] = rc->Rg[j - 1] + range_panel(m, rc->E[j - 1], rc->E[j]);
    }
    rc->E[OR_RG_LATTICE - 1] = e_max;
}

/* R_g(E) if it can be <= limit, else a value > limit (the exact integral is
 * computed whenever it matters; the cache only rules out large ranges). */
static double residual_range_g(const or_material* m, const range_cache* rc, double E,
                               double limit) {
    int j = (int)floor((log(E) - rc->lnlo) / rc->dln);
    if (j < 0) j = 0;
    if (j > OR_RG_LATTICE - 2) j = OR_RG_LATTICE - 2;
    while (j > 0 && rc->E[j] > E) --j;
    while (j < OR_RG_LATTICE - 2 && rc->E[j + 1] <= E) ++j;
    if (rc->Rg[j] > limit) return rc->Rg[j];
    return rc->Rg[j] + range_panel(m, rc->E[j], E);
}

/* Exported: exact CSDA range in g/cm^2 and stopping power, for the pins. */
double or_csda_range_g(const or_material* m, double e_min, double E) {
    gl_init();
    /* panels uniform in ln E, fine enough for 1e-13 relative accuracy */
    int np = 2048;
    double a = log(e_min), b = log(E), s = 0.0;
    for (int k = 0; k < np; ++k) {
        double lo = exp(a + (b - a) * k / np), hi = exp(a + (b - a) * (k + 1) / np);
        s += range_panel(m, lo, hi);
    }
    return s;
}
double or_stopping_mass(const or_material* m, double E) { return stopping_mass(m, E); }
double or_straggle_mass(const or_material* m, double E) { return straggle_mass(m, E); }
double or_ld_sigma(const or_material* m, double rho, double E, double z, double F) {
    return lynch_dahl_sigma(m, rho, E, z, F);
}
double or_rutherford_integral_barn(double Z, double A, double E, double tc) {
    return rutherford_integral_barn(Z, A, E, tc);
}
double or_mott_integral_barn(double A, double E, double tc, double tb) {
    return mott_integral_barn(A, E, tc, tb);
}
double or_mott_G(double eta, double mu) { return mott_G(eta, mu); }
double or_mott_eta(double E) { return mott_eta(E); }
double or_eta2_over_k2_fm2(double Z, double A, double E) { return eta2_over_k2_fm2(Z, A, E); }
double or_rutherford_one_minus_mu(double U, double tc) { return rutherford_one_minus_mu(U, tc); }
double or_mott_sample_mu(double E, double U, double tc, double tb) {
    return mott_sample_mu(E, U, tc, tb);
}
double or_kalbach_mu(double a, double r, double U) { return kalbach_mu(a, r, U); }
double or_cm_to_lab(double K, double A, double c, double s, double u) {
    return cm_to_lab(K, A, c, s, u);
}
void or_turn(double* d, double ct, double st, double phi) { turn(d, ct, st, phi); }
double or_sbm_lineage_mean(double t) { return sbm_lineage_mean(t); }
double or_sbm_lineage_var(double t) { return sbm_lineage_var(t); }
double or_sbm_upper_tail(double t, double c) { return sbm_upper_tail(t, c); }
double or_sbm_t_switch(void) { return SBM_T_SWITCH; }
void or_sbm_polar_n(size_t n, double t, const double* z, const double* u, double* ct, double* st) {
    for (size_t i = 0; i < n; ++i) sbm_polar(t, z[i], u[i], &ct[i], &st[i]);
}
/* Inelastic-branch pieces, exported for the pins. */
void or_lattice_pos(const or_nuclear* nu, double E, int* i, double* f) { lattice_pos(nu, E, i, f); }
double or_inelastic_sigma_barn(const or_nuclear* nu, int t, double E) {
    return inelastic_sigma_barn(nu, t, E);
}
void or_inelastic_draw(const or_nuclear* nu, int t, double E, double U1, double U3,
                       double* u_loss, double* cos_cm) {
    inelastic_draw(nu, t, E, U1, U3, u_loss, cos_cm);
}
/* which: 0 = loss-fraction inverse CDF, 1 = Kalbach r, 2 = Kalbach a */
double or_table_eu(const or_nuclear* nu, int t, int which, double E, double x) {
    const double* base = which == 0 ? nu->u_icdf : which == 1 ? nu->kr : nu->ka;
    return table_eu(nu, base + (size_t)t * nu->n_e * nu->n_u, E, x);
}
double or_bspline3(const double* c, int m, double x0, double h, double x) {
    return bspline3(c, m, x0, h, x);
}
double or_p_ni_integral(const or_nuclear* nu, int t, int i, double x) {
    return p_ni_integral(nu, t, i, x);
}
double or_ni_density(const or_nuclear* nu, int t, double E, double mu) {
    return ni_density(nu, t, E, mu);
}
double or_ni_integral(const or_nuclear* nu, int t, double E, double x) {
    return ni_integral(nu, t, E, x);
}
double or_h_nuclear_density(const or_nuclear* nu, double E, double mu) {
    return h_nuclear_density(nu, E, mu);
}
double or_h_nuclear_antiderivative(const or_nuclear* nu, double E, double mu) {
    return h_nuclear_antiderivative(nu, E, mu);
}
double or_elastic_sample_mu(const or_nuclear* nu, int Z, double A, double E, double U,
                            double tc, double tb) {
    return elastic_sample_mu(nu, Z, A, E, U, tc, tb);
}
double or_elastic_cum_barn(const or_nuclear* nu, int Z, double A, double E, double lo, double x) {
    return elastic_cum_barn(nu, Z, A, E, lo, x);
}
double or_elastic_cut(const or_material* m, const or_params* p, double rho, double E) {
    return elastic_cut(m, p, rho, E);
}
double or_channel_total_rate(const or_material* m, const or_nuclear* nu, const or_params* p,
                             double rho, double E) {
    channels c;
    channel_rates(m, nu, p, rho, E, &c);
    double s = 0.0;
    for (int k = 0; k < c.n; ++k) s += c.rate[k];
    return s;
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */

/* D is closed: a point is inside iff every coordinate lies in [lo, hi]. */
static int inside(const or_phantom* ph, const double r[3]) {
    const int n[3] = {ph->nx, ph->ny, ph->nz};
    for (int k = 0; k < 3; ++k) {
        double lo = ph->origin[k], hi = ph->origin[k] + n[k] * ph->d[k];
        if (!(r[k] >= lo && r[k] <= hi)) return 0;
    }
    return 1;
}

/* Voxel of an inside point; the upper face belongs to the last voxel. */
static size_t voxel(const or_phantom* ph, const double r[3]) {
    const int n[3] = {ph->nx, ph->ny, ph->nz};
    int i[3];
    for (int k = 0; k < 3; ++k) {
        int v = (int)floor((r[k] - ph->origin[k]) / ph->d[k]);
        if (v < 0) v = 0;
        if (v > n[k] - 1) v = n[k] - 1;
        i[k] = v;
    }
    return ((size_t)i[2] * ph->ny + i[1]) * ph->nx + i[0];
}

/* ------------------------------------------------------------------------ */
/* Transport                                                                  */
/* ------------------------------------------------------------------------ */

/* Ledger slots */
enum { L_DEP = 0, L_ESC, L_NUC, L_E0, L_TRUNC, L_STEPS, L_HIST, L_JUMPS, L_N };
/* Per-history record fields */
enum { R_E0 = 0, R_DEP, R_ESC, R_NUC, R_TRUNC, R_STEPS, R_NEL, R_NNE, R_END,
       R_X, R_Y, R_Z, R_OX, R_OY, R_OZ, R_EEND, R_J1, R_J2, R_N };
/* End codes */
enum { END_EOR = 1, END_EXIT = 2, END_EMIN = 3, END_MAXSTEPS = 4, END_SOURCE = 5 };

typedef struct {
    double* edep;    /* weighted energy per voxel, or NULL */
    double hist[R_N];
    double wgt;
} score_ctx;

static void deposit(const or_phantom* ph, score_ctx* sc, const double at[3], double e) {
    if (inside(ph, at)) {
        if (sc->edep) sc->edep[voxel(ph, at)] += sc->wgt * e;
        sc->hist[R_DEP] += e;
    } else {
        sc->hist[R_ESC] += e;
    }
}

/* Source of history h (the workloads' Gaussian pencil beam; the paper's
 * own beam is a monoenergetic nozzle, section 2.2.2): energy
 * E_s (1 + sigma_E Z3) and lateral position (x_s, y_s) + sigma_xy (Z1, Z2)
 * on the entrance face z0, direction +z.  Block (h, 2^32-1, 0): the
 * Box-Muller pair (cos, sin) of (w0, w1) gives Z1, Z2, and (w2, w3) gives
 * Z3 by its cosine. */
static void source(const or_spot* sp, double z0, uint64_t seed, uint64_t h, double* E,
                   double R[3]) {
    uint32_t w[4];
    rng_block(seed, h, 0xFFFFFFFFu, 0, w);
    double rr = sqrt(-2.0 * log(u_hi(w[0])));
    double z1 = rr * cos(TWO_PI * u_hi(w[1])), z2 = rr * sin(TWO_PI * u_hi(w[1]));
    double z3 = sqrt(-2.0 * log(u_hi(w[2]))) * cos(TWO_PI * u_hi(w[3]));
    *E = sp->E * (1.0 + sp->sigmaE * z3);
    R[0] = sp->x + sp->sigma_xy * z1;
    R[1] = sp->y + sp->sigma_xy * z2;
    R[2] = z0;
}

/* Exported for the pins: source energy and position of histories
 * [h0, h0 + n) of one spot; out is n x 4 (E, x, y, z). */
void or_source_n(const or_spot* sp, double z0, uint64_t seed, uint64_t h0, size_t n,
                 double* out) {
    for (size_t i = 0; i < n; ++i) source(sp, z0, seed, h0 + i, &out[4 * i], &out[4 * i + 1]);
}

/* One sequential proton track, Eq. (VSDE) with the jump law of Eq. (Npi),
 * until it leaves D, falls below e_min, or ends its range.  Coefficients
 * are taken at Y_n: the material and density of the voxel holding R_n and
 * the energy E_n. */
static void track(const or_material* mats, const range_cache* rcs, const or_params* p,
                  const or_nuclear* nu, const or_phantom* ph, const or_spot* sp,
                  uint64_t seed, uint64_t h, score_ctx* sc) {
    const double D = p->step_cm;
    uint32_t w[4];

    double E, R[3];
    source(sp, ph->origin[2], seed, h, &E, R);
    double O[3] = {0.0, 0.0, 1.0};
    sc->hist[R_E0] = E;

    int end = 0;
    long long n = 0;
    double e_end = E;
    sc->hist[R_J1] = -1.0;
    sc->hist[R_J2] = -1.0;
    if (!inside(ph, R)) {
        sc->hist[R_ESC] += E; E = 0.0; end = END_SOURCE;
    } else if (E < p->e_min) {
        deposit(ph, sc, R, E); E = 0.0; end = END_SOURCE;
    }

    while (!end) {
        e_end = E;
        if (n >= p->max_steps) { sc->hist[R_TRUNC] += E; end = END_MAXSTEPS; break; }
        size_t v = voxel(ph, R);
        const or_material* m = &mats[ph->mat[v]];
        double rho = (double)ph->rho[v];

        /* End of range: when the residual CSDA range at E_n fits in one
         * step, move it and deposit all of E_n at its midpoint. */
        if (p->flags & OR_EOR) {
            double rg = residual_range_g(m, &rcs[ph->mat[v]], E, D * rho);
            double rres = rg / rho;
            if (rres <= D) {
                double mid[3], fin[3];
                for (int k = 0; k < 3; ++k) {
                    mid[k] = R[k] + O[k] * 0.5 * rres;
                    fin[k] = R[k] + O[k] * rres;
                }
                deposit(ph, sc, mid, E);
                memcpy(R, fin, sizeof R);
                E = 0.0; end = END_EOR; n++;
                break;
            }
        }

        rng_block(seed, h, (uint32_t)n, 0, w);

        /* Continuous loss with clamped straggling, first line of Eq. (VSDE). */
        double s1 = (p->flags & OR_LOSS) ? rho * stopping_mass(m, E) : 0.0;
        double X = 0.0;
        if (p->flags & OR_STRAGGLE) {
            double s2 = sqrt(rho * straggle_mass(m, E));
            double zE = sqrt(-2.0 * log(u_hi(w[0]))) * cos(TWO_PI * u_hi(w[1]));
            X = s2 * sqrt(D) * zE;      /* B_n ~ N(0, Delta) */
            if (X < -s1 * D) X = -s1 * D;
            if (X > s1 * D) X = s1 * D;
        }
        double Ep = E - s1 * D + X;
        if (Ep < 0.0) Ep = 0.0;

        /* Jump: none with probability exp(-Delta sum sigma), else one event
         * from the mixture Eq. (Npi) (elastic: u = 0; inelastic: u from pi_ne). */
        double u_loss = 0.0;
        int jumped = 0;
        double jc = 1.0, js = 0.0, jphi = 0.0;
        if (p->flags & (OR_ELASTIC | OR_INELASTIC)) {
            channels ch;
            channel_rates(m, nu, p, rho, E, &ch);
            double tot = 0.0;
            for (int k = 0; k < ch.n; ++k) tot += ch.rate[k];
            double pj = -expm1(-D * tot);
            if (tot > 0.0 && u_lo(w[0], w[1], w[2]) < pj) {
                uint32_t q[4];
                rng_block(seed, h, (uint32_t)n, 1, q);
                double t = u_hi(q[0]) * tot, acc = 0.0;
                int c = ch.n - 1;
                for (int k = 0; k < ch.n; ++k) {
                    acc += ch.rate[k];
                    if (t < acc) { c = k; break; }
                }
                int e = ch.elem[c];
                double cos_cm, sin_cm;
                if (!ch.inel[c]) {
                    double tc = cut_for(m->Z[e], ch.theta_c, p->theta_bs);
                    if (elastic_nuclear_integral_barn(nu, m->Z[e], E, tc, p->theta_bs) != 0.0) {
                        cos_cm = elastic_sample_mu(nu, m->Z[e], m->A[e], E, u_hi(q[1]), tc,
                                                   p->theta_bs);
                        sin_cm = sqrt(fmax(0.0, 1.0 - cos_cm * cos_cm));
                    } else if (m->Z[e] == 1) {
                        cos_cm = mott_sample_mu(E, u_hi(q[1]), tc, p->theta_bs);
                        sin_cm = sqrt(fmax(0.0, 1.0 - cos_cm * cos_cm));
                    } else {
                        double om = rutherford_one_minus_mu(u_hi(q[1]), tc);
                        cos_cm = 1.0 - om;
                        sin_cm = sqrt(om * (2.0 - om));
                    }
                    sc->hist[R_NEL] += 1.0;
                } else {
                    inelastic_draw(nu, ch.tab[c], E, u_hi(q[1]), u_hi(q[3]), &u_loss, &cos_cm);
                    sin_cm = sqrt(fmax(0.0, 1.0 - cos_cm * cos_cm));
                    sc->hist[R_NNE] += 1.0;
                }
                double thl = cm_to_lab(E, m->A[e], cos_cm, sin_cm, u_loss);
                jc = cos(thl); js = sin(thl);
                jphi = TWO_PI * u_hi(q[2]);
                jumped = 1;
                if (sc->hist[R_J1] < 0.0) sc->hist[R_J1] = (double)n;
                sc->hist[R_J2] = (double)n;
            }
        }
        double En = Ep * (1.0 - u_loss);
        sc->hist[R_NUC] += Ep - En;

        /* Energy E_n - E' is deposited at the step midpoint. */
        double mid[3], Rn[3];
        for (int k = 0; k < 3; ++k) {
            mid[k] = R[k] + O[k] * 0.5 * D;
            Rn[k] = R[k] + O[k] * D;
        }
        deposit(ph, sc, mid, E - Ep);

        /* Direction: small-angle diffusion, then the jump, then renormalise. */
        if (p->flags & OR_MCS) {
            double sig = lynch_dahl_sigma(m, rho, E, p->ld_z_cm, p->ld_F) * sqrt(D / p->ld_z_cm);
            if (p->flags & OR_SBM) {
                /* the lineage count's normal: the sine partner of Z_E's Box-Muller pair */
                double zM = sqrt(-2.0 * log(u_hi(w[0]))) * sin(TWO_PI * u_hi(w[1]));
                double ct, st;
                sbm_polar(sig * sig, zM, u_hi(w[2]), &ct, &st);
                turn(O, ct, st, TWO_PI * u_hi(w[3]));
            } else {
                geodesic_step(O, sig, u_hi(w[2]), u_hi(w[3]));
            }
        }
        if (jumped) turn(O, jc, js, jphi);
        normalize(O);

        memcpy(R, Rn, sizeof R);
        E = En;
        n++;
        e_end = E;
        if (!inside(ph, R)) { sc->hist[R_ESC] += E; E = 0.0; end = END_EXIT; break; }
        if (E < p->e_min) { deposit(ph, sc, R, E); E = 0.0; end = END_EMIN; break; }
    }
    sc->hist[R_STEPS] = (double)n;
    sc->hist[R_END] = end;
    sc->hist[R_X] = R[0]; sc->hist[R_Y] = R[1]; sc->hist[R_Z] = R[2];
    sc->hist[R_OX] = O[0]; sc->hist[R_OY] = O[1]; sc->hist[R_OZ] = O[2];
    sc->hist[R_EEND] = e_end;
}

/* Transport histories [h_begin, h_end) of the spot list.  History h belongs
 * to the spot whose cumulative count range holds it and carries weight
 * weight/n of that spot.  edep (nvox doubles, may be NULL) receives the
 * weighted deposited energy in MeV; ledger[8] the weighted energy balance
 * and counts; records ((h_end-h_begin) x 18, may be NULL) per-history data
 * (R_EEND: energy at the end event, before absorption; R_J1, R_J2: first and
 * last jump step, -1 if none).
 * Returns 0, or -1 on invalid input. */
int or_transport(const or_material* mats, int n_mat, const or_params* p, const or_nuclear* nu,
                 const or_phantom* ph, const or_spot* spots, int n_spots, uint64_t seed,
                 uint64_t h_begin, uint64_t h_end, int n_threads, double* edep,
                 double* ledger, double* records) {
    if (n_mat < 1 || n_mat > OR_MAX_MAT || n_spots < 1 || h_end < h_begin) return -1;
    gl_init();
    for (int k = 0; k < n_mat; ++k)
        if (!(stopping_mass(&mats[k], p->e_min) > 0.0)) return -1;
    range_cache* rcs = (range_cache*)malloc(sizeof(range_cache) * n_mat);
    if (!rcs) return -1;
    for (int k = 0; k < n_mat; ++k) range_cache_init(&mats[k], p->e_min, p->e_max, &rcs[k]);

    uint64_t* pre = (uint64_t*)malloc(sizeof(uint64_t) * (n_spots + 1));
    pre[0] = 0;
    for (int s = 0; s < n_spots; ++s) pre[s + 1] = pre[s] + spots[s].n;

    size_t nvox = (size_t)ph->nx * ph->ny * ph->nz;
    double led[L_N] = {0};
    int nt = n_threads > 0 ? n_threads : 1;
#ifndef _OPENMP
    nt = 1;
#endif
    double** part = (double**)calloc(nt, sizeof(double*));
    double* pled = (double*)calloc((size_t)nt * L_N, sizeof(double));

#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* mine = NULL;
        if (edep) {
            mine = (tid == 0) ? edep : (double*)calloc(nvox, sizeof(double));
            part[tid] = mine;
        }
        double* ml = pled + (size_t)tid * L_N;
#pragma omp for schedule(dynamic, 64)
        for (long long hh = (long long)h_begin; hh < (long long)h_end; ++hh) {
            uint64_t h = (uint64_t)hh;
            int s = 0;
            while (s < n_spots - 1 && h >= pre[s + 1]) ++s;
            score_ctx sc;
            memset(&sc, 0, sizeof sc);
            sc.edep = mine;
            sc.wgt = spots[s].weight / (double)spots[s].n;
            track(mats, rcs, p, nu, ph, &spots[s], seed, h, &sc);
            ml[L_DEP] += sc.wgt * sc.hist[R_DEP];
            ml[L_ESC] += sc.wgt * sc.hist[R_ESC];
            ml[L_NUC] += sc.wgt * sc.hist[R_NUC];
            ml[L_E0] += sc.wgt * sc.hist[R_E0];
            ml[L_TRUNC] += sc.wgt * sc.hist[R_TRUNC];
            ml[L_STEPS] += sc.hist[R_STEPS];
            ml[L_HIST] += 1.0;
            ml[L_JUMPS] += sc.hist[R_NEL] + sc.hist[R_NNE];
            if (records) memcpy(records + (size_t)(h - h_begin) * R_N, sc.hist, sizeof sc.hist);
        }
    }
    /* fixed-order reduction */
    if (edep) {
        for (int t = 1; t < nt; ++t) {
            if (!part[t]) continue;
            for (size_t i = 0; i < nvox; ++i) edep[i] += part[t][i];
            free(part[t]);
        }
    }
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < L_N; ++k) led[k] += pled[(size_t)t * L_N + k];
    if (ledger) for (int k = 0; k < L_N; ++k) ledger[k] += led[k];
    free(part); free(pled); free(pre); free(rcs);
    return 0;
}

/* Dose to medium in Gy: E (MeV) / (rho V), section 2.2 ("Test cases"). */
void or_dose(const double* edep, const float* rho, size_t nvox, double voxel_cm3, double* dose) {
    for (size_t i = 0; i < nvox; ++i)
        dose[i] = rho[i] > 0.0f ? edep[i] * MEV_TO_J / ((double)rho[i] * voxel_cm3 * 1e-3) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Gamma index (section 2.2, "Comparison metrics"): for each reference      */
/* voxel with dose >= thresh * max(ref), gamma = min over points x within   */
/* the distance-to-agreement of sqrt(|x-r|^2/DTA^2 + (De(x)-Dr)^2/(DD n)^2) */
/* with n = Dr (local) or max(ref) (global); De is trilinear in the         */
/* evaluated grid; x runs over the lattice of spacing DTA/interp around r. */
/* Returns the pass fraction; n_eval/n_pass get the counts.                 */
/* ------------------------------------------------------------------------ */
static double trilinear(const double* g, int nx, int ny, int nz, double fx, double fy,
                        double fz, int* ok) {
    if (fx < 0.0 || fy < 0.0 || fz < 0.0 || fx > nx - 1 || fy > ny - 1 || fz > nz - 1) {
        *ok = 0;
        return 0.0;
    }
    int ix = (int)floor(fx), iy = (int)floor(fy), iz = (int)floor(fz);
    if (ix > nx - 2) ix = nx > 1 ? nx - 2 : 0;
    if (iy > ny - 2) iy = ny > 1 ? ny - 2 : 0;
    if (iz > nz - 2) iz = nz > 1 ? nz - 2 : 0;
    double tx = fx - ix, ty = fy - iy, tz = fz - iz;
    int jx = nx > 1 ? ix + 1 : ix, jy = ny > 1 ? iy + 1 : iy, jz = nz > 1 ? iz + 1 : iz;
#define G(a, b, c) g[((size_t)(c) * ny + (b)) * nx + (a)]
    double c00 = G(ix, iy, iz) * (1 - tx) + G(jx, iy, iz) * tx;
    double c10 = G(ix, jy, iz) * (1 - tx) + G(jx, jy, iz) * tx;
    double c01 = G(ix, iy, jz) * (1 - tx) + G(jx, iy, jz) * tx;
    double c11 = G(ix, jy, jz) * (1 - tx) + G(jx, jy, jz) * tx;
#undef G
    double c0 = c00 * (1 - ty) + c10 * ty, c1 = c01 * (1 - ty) + c11 * ty;
    *ok = 1;
    return c0 * (1 - tz) + c1 * tz;
}

static int cmp_r2(const void* a, const void* b) {
    double x = ((const double*)a)[3], y = ((const double*)b)[3];
    return (x > y) - (x < y);
}

double or_gamma(const double* ref, const double* ev, int nx, int ny, int nz, const double* d,
                double dd, double dta, double thresh, int interp, int local, int n_threads,
                long long* n_eval, long long* n_pass) {
    size_t nvox = (size_t)nx * ny * nz;
    double mx = 0.0;
    for (size_t i = 0; i < nvox; ++i) if (ref[i] > mx) mx = ref[i];
    double step = dta / interp;
    int K = interp;
    int cap = (2 * K + 1) * (2 * K + 1) * (2 * K + 1);
    double* off = (double*)malloc(sizeof(double) * 4 * cap);
    int no = 0;
    for (int a = -K; a <= K; ++a)
        for (int b = -K; b <= K; ++b)
            for (int c = -K; c <= K; ++c) {
                double ox = a * step, oy = b * step, oz = c * step;
                double r2 = ox * ox + oy * oy + oz * oz;
                if (r2 <= dta * dta * (1.0 + 1e-12)) {
                    off[4 * no] = ox; off[4 * no + 1] = oy; off[4 * no + 2] = oz;
                    off[4 * no + 3] = r2;
                    no++;
                }
            }
    /* nearest points first, so a passing voxel stops early */
    qsort(off, no, 4 * sizeof(double), cmp_r2);
    long long ne = 0, np = 0;
    int nt = n_threads > 0 ? n_threads : 1;
#pragma omp parallel for num_threads(nt) reduction(+ : ne, np) schedule(dynamic, 256)
    for (long long i = 0; i < (long long)nvox; ++i) {
        double dr = ref[i];
        if (!(dr >= thresh * mx) || dr <= 0.0) continue;
        ne++;
        int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((size_t)nx * ny));
        double norm = dd * (local ? dr : mx);
        int pass = 0;
        for (int k = 0; k < no && !pass; ++k) {
            int ok;
            double de = trilinear(ev, nx, ny, nz, ix + off[4 * k] / d[0],
                                  iy + off[4 * k + 1] / d[1], iz + off[4 * k + 2] / d[2], &ok);
            if (!ok) continue;
            double g2 = off[4 * k + 3] / (dta * dta) + (de - dr) * (de - dr) / (norm * norm);
            if (g2 <= 1.0) pass = 1;
        }
        np += pass;
    }
    free(off);
    if (n_eval) *n_eval = ne;
    if (n_pass) *n_pass = np;
    return ne ? (double)np / (double)ne : 1.0;
}

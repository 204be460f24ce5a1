// Internal layouts shared by the host side of libsde and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sde {

constexpr int kMaxElem = 16;
constexpr int kMaxMat = 8;
constexpr int kLedgerN = 9;

// Physical constants (CODATA 2018), MeV based.
constexpr double kMp = 938.27208816;       // proton rest energy
constexpr double kMe = 0.51099895000;      // electron rest energy
constexpr double kAlpha = 7.2973525693e-3;
constexpr double kNa = 6.02214076e23;
constexpr double kHbarcFm = 197.3269804;   // MeV fm
constexpr double kAmu = 931.49410242;      // MeV
constexpr double kMevToJ = 1.602176634e-13;
constexpr double kBethe = 0.3072;          // Eq. (bethbloch) constant, MeV cm^2/mol
constexpr double kBoxMullerMax = 5.77;     // |Z| bound of a 23-bit Box-Muller draw

// One element of a medium, read only inside the (rare) jump branch.
struct ElemDev {
    float Z;
    float m2;        // target rest energy A * amu, MeV
    float el_coef;   // elastic rate = rho * el_coef / E^2 (times the Mott bracket for H)
    float ne_coef;   // inelastic rate = rho * ne_coef * sigma_barn(E)
    int is_h;        // hydrogen: Mott (identical-particle) cross section
    int tab;         // row of the inelastic tables, -1 if none
    float el_base;   // el_coef without the cut's factor (T - 1/2 for Rutherford; = el_coef for H)
    int ni;          // row of the sigma_NI P_NI tables, -1 if none (hydrogen: -1)
    float nuc_coef;  // 2 pi N_A w / A 1e-24: nuclear elastic rate / rho per barn of integral
    int hn;          // hydrogen with partial-wave amplitudes
    int pad2, pad3;
};

struct MatDev {
    float zoa;             // sum_i w_i Z_i / A_i
    float log_pre;         // ln(2 m_e / I) - 2 ln(m_p): Bethe log = log_pre + ln(p^2) - beta^2
    int n_elem;
    int pad;
    float c_ruth;          // sum of non-hydrogen el_coef: Rutherford rate = rho c_ruth / E^2
    float c_mott;          // hydrogen el_coef: Mott rate = rho c_mott / E^2 * bracket(E)
    float c_ruth0;         // c_ruth without the cut's factor T - 1/2
    float pad2;
    ElemDev el[kMaxElem];
};

// The same medium in double precision, for the FP64 instance of the
// transport: Bethe and Lynch-Dahl constants per element (the small-angle
// width is evaluated from its formula there, not from the lattice table)
// and the jump constants.
struct MatDev64 {
    double zoa, log_pre;   // as in MatDev
    double c_ruth, c_mott, c_ruth0;   // as in MatDev
    int n_elem, pad[3];
    double wz[kMaxElem];      // w_i Z_i (Z_i + 1) / A_i
    double ln_ca[kMaxElem];   // ln(2.007e-5 Z_i^(2/3))
    double za2[kMaxElem];     // 3.34 (Z_i alpha)^2
    double el_coef[kMaxElem], el_base[kMaxElem], ne_coef[kMaxElem], m2[kMaxElem];
    double nuc_coef[kMaxElem];
    int is_h[kMaxElem], tab[kMaxElem], ni[kMaxElem], hn[kMaxElem];
};

// Per-spot source data on the device in the stepping precision R.
// wscale = weight / n * 2^k.
template <class R>
struct SpotT {
    R E, sigmaE, x, y, sxy, wscale;
    unsigned long long h0;   // index of the spot's first history in the caller's order
};
using SpotDev = SpotT<float>;
using SpotDev64 = SpotT<double>;

// Scheme and geometry scalars in the stepping precision R.
template <class R>
struct KScal {
    R step, half_step, sqrt_step, e_min;
    R c_bethe, c_strag;              // 0.3072, 4 pi N_A (alpha hbar c)^2
    R ruth_T;                        // 1 / (1 - cos theta_cut)
    R mott_lo, mott_hi;              // CM cosine limits of hydrogen elastic
    R mott_D0, mott_Lhi, mott_Llo;   // bracket terms at the fixed cut
    R mott_Dlo;                      // 2 lo / (1 - lo^2), the bracket's lower rational term
    R mott_shi, mott_slo;            // 1 - hi (fixed cut) and 1 - lo
    R z_over_step;                   // ld_z / step
    R eta_pre;                       // alpha sqrt(m_p / 2): eta = eta_pre / sqrt(E)
    R ln_e_lo, inv_dln;              // lattice: t = (ln E - ln_e_lo) inv_dln
    R ld_z, ld_F;                    // Lynch-Dahl path length and central fraction
    R lo[3], hi[3], inv_d[3], d[3];  // phantom box and voxel size
};

// Everything the transport kernel reads; passed by value.
struct KParams {
    // tables
    const float4* hot;         // [n_mat][n_e] {A1, A2, inelastic rate/rho, elastic rate E^2/rho}
    const double2* rg64;       // [n_mat][n_e] {Rg, dRg/dt} for the FP64 end of range
    const MatDev* mats;        // [n_mat]
    const float* nuc_sigma;    // [n_tab][n_e] barn
    const float* nuc_u;        // [n_tab][n_e][n_u]
    const float* nuc_r;
    const float* nuc_a;
    int n_mat, n_e, n_u, n_tab;
    // tables of the FP64 instance
    const MatDev64* mats64;          // [n_mat]
    const double2* hot64;            // [n_mat][n_e] {inelastic rate/rho, elastic rate E^2/rho}
    const double* nuc_sigma64;       // the nuclear tables unrounded
    const double* nuc_u64;
    const double* nuc_r64;
    const double* nuc_a64;
    // elastic nuclear data (section 2.1.4): sigma_NI P_NI splines in mu per
    // lattice energy, with their cumulative integrals at the knots
    // ([n_ni][n_e][n_mu - 2]), and hydrogen's amplitude splines in the
    // lattice coordinate ([3][n_l][n_e + 2]: Re a_l, Im a_l, b_l)
    int n_ni, n_mu, n_l, pad7;
    const float* ni_p;
    const float* ni_cum;
    const float* ni_sig;
    const double* ni_p64;
    const double* ni_cum64;
    const double* ni_sig64;
    const double* h_coef;
    // scheme and geometry scalars per precision
    KScal<float> sf;
    KScal<double> sd;
    unsigned flags;                  // physics switches (SDE_ALL bits)
    int fp64;                        // step in double precision
    long long max_steps;
    // phantom
    const uint2* vox;                // [nz][ny][nx] {density bits, material}
    int nx, ny, nz, pad1;
    // beam
    const SpotDev* spots;
    const SpotDev64* spots64;        // the same spots in double precision
    const unsigned long long* prefix;   // [n_spots + 1] cumulative history counts, claim order
    int n_spots, pad3;
    unsigned long long n_hist;
    unsigned long long seed;
    // outputs and work queue
    unsigned long long* tally;       // [n_rep][nvox] fixed point, one replica per XCD
    unsigned long long rep_stride;   // nvox
    int n_rep, pad6;
    unsigned long long* ledger;      // [kLedgerN]
    unsigned long long* counter;     // next history
    float* rec;                      // optional [n_hist][12] per-history records
    float ec[kMaxMat];               // end-of-range screen energy per material (this phantom)
    int jump_batch;                  // finish pending jumps when this many lanes wait
    int claim_chunk;                 // history indices a wave takes from the counter at once
    int refill;
    int tile_nx, tile_ny, tile_nz, tile_x0, tile_y0, tile_z0, pad4;
    unsigned long long nan_h;        // test hook: this history starts with a NaN direction
};

// Launchers (sde_kernels.hip)
hipError_t launch_pack_phantom(const uint8_t* mat, const float* rho, uint2* vox, size_t nvox,
                               int n_mat, unsigned int* bad, unsigned int* rho_max_bits,
                               hipStream_t s);
hipError_t launch_reset(unsigned long long* tally, size_t n, unsigned long long* ledger,
                        unsigned long long* counter, hipStream_t s);
hipError_t launch_transport(const KParams& p, int grid, int block, size_t lds_bytes,
                            hipStream_t s);
hipError_t launch_convert(unsigned long long* tally, int n_rep, const uint2* vox, size_t nvox,
                          double inv_scale, double voxel_cm3, double* dose,
                          unsigned long long* ledger, hipStream_t s);
// gamma_kernels.hip: offsets on the lattice of spacing dta / interp
// (interp <= 50) within dta; use_bound needs dta below a voxel on every axis.
// counts[4] = {evaluated, passed, maximum bits, list length} (counts[0], [1]
// and [3] zero on entry); list: cap voxel indices of scratch.
hipError_t launch_gamma(const double* ref, const double* ev, int nx, int ny, int nz, int interp,
                        double dta, double dx, double dy, double dz, double dd, double thr_abs,
                        double max_ref, int local, int use_bound, unsigned long long* counts,
                        unsigned* list, unsigned cap, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
hipError_t launch_max(const double* a, size_t n, unsigned long long* out_bits, hipStream_t s);
hipError_t launch_sbm_polar(const float* t, const float* u, const float* z, int n, float* c,
                            float* s_out, hipStream_t s);
hipError_t transport_kernel_attributes(size_t lds_bytes);
hipError_t launch_philox_words(unsigned long long seed, const unsigned long long* h,
                               const unsigned* n, const unsigned* b, int count, uint4* out,
                               hipStream_t s);

}  // namespace sde

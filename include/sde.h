/*
 * libsde: MI355X (gfx950) jump-SDE proton dose engine, C ABI.
 *
 * Method: Dean et al., "SDE-based Monte Carlo dose calculation for proton
 * therapy validated against Geant4" (arXiv 2511.03115).  Each proton history
 * follows the Euler-Maruyama scheme of section 2.1.2, Eq. (VSDE): Bethe-Bloch
 * continuous loss (Eq. (bethbloch), Bragg additivity) with clamped straggling
 * (Eq. (energystraggling)), Lynch-Dahl small-angle diffusion on the sphere
 * (section 2.1.4), and Poisson-clocked large-angle elastic and inelastic
 * nuclear jumps (Eq. (Npi), sections 2.1.4-2.1.5, Appendix A.1).  Energy
 * E_n - E' is scored at each step midpoint into an int64 fixed-point voxel
 * tally and converted to dose-to-medium (section 2.2.2).
 *
 * Conventions
 *  - Every function returns 0 (SDE_OK) or a negative sde_status; no C++
 *    exception crosses this boundary.  sde_last_error() gives a message for
 *    the last failure on the calling thread.
 *  - Host pointers are marked (host), device pointers (device).  The caller
 *    owns every argument array; the library owns its tables, tally and work
 *    counters and releases them in sde_free().
 *  - Work is enqueued on the stream set by sde_set_stream (default: the null
 *    stream) and is complete when that stream is synchronised.  The library
 *    keeps global state: calls must not overlap from several host threads.
 *  - Units: MeV, cm, g/cm^3, Gy.  Voxel arrays are C-contiguous
 *    [nz][ny][nx] (x fastest); the beam enters through the low-z face along +z.
 *  - Results are a pure function of (materials, params, nuclear tables,
 *    beam, phantom, history count, seed): bit-identical across runs and
 *    launch configurations (integer tally, counter-based RNG keyed by
 *    (seed, history, step)).  History h is the h-th history in the order
 *    of the beam's spots (spot i owns the n_i indices after those of spots
 *    0..i-1), whatever order the kernel runs them in.
 */
#ifndef SDE_H
#define SDE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SDE_OK = 0,
    SDE_E_INVALID = -1,   /* bad argument or descriptor */
    SDE_E_HIP = -2,       /* HIP runtime error */
    SDE_E_RANGE = -3,     /* a beam energy outside [e_min, e_max] of the tables */
    SDE_E_OVERFLOW = -4,  /* the fixed-point tally could overflow */
    SDE_E_STATE = -5,     /* called before sde_init_materials */
    SDE_E_NOMEM = -6      /* allocation failed */
} sde_status;

#define SDE_MAX_ELEM 16   /* elements per material */
#define SDE_MAX_MAT 8     /* materials per phantom (LDS table budget) */

/* Physics switches (sde_physics_params.flags).  SDE_ALL is the method;
 * bits other than these, SDE_FP64 and SDE_ECUT are rejected. */
#define SDE_LOSS 1u          /* continuous loss, Eq. (bethbloch) */
#define SDE_STRAGGLE 2u      /* straggling noise, Eq. (energystraggling) */
#define SDE_MCS 4u           /* small-angle diffusion on S^2 */
#define SDE_ELASTIC 8u       /* large-angle elastic jumps */
#define SDE_INELASTIC 16u    /* inelastic nuclear jumps */
#define SDE_END_OF_RANGE 32u /* residual-range final step near the Bragg peak */
/* With SDE_MCS: draw the small-angle diffusion from the spherical Brownian
 * motion law at time t = sigma^2 Delta / z (section 2.2.2; the cited
 * Algorithm 1 of Mijatovic et al. with Griffiths' normal lineage count for
 * t < 0.02, exact inversion of the heat kernel's Legendre series above).
 * Without it, the geodesic Gaussian step of per-axis variance t (O(t)
 * from that law in the angle; ~2 % less time on a 150 MeV water beam). */
#define SDE_SBM 64u
#define SDE_ALL 127u
/* Not a physics switch: step in double precision.  The same kernel source
 * instantiated on double, with the Lynch-Dahl width and the elastic jump
 * rate evaluated from their formulas at each step instead of interpolated
 * from the FP32 lattice tables (section 2.1.4), so that histories follow a
 * double-precision reference step by step; for checks against such a
 * reference, several times slower than the default single-precision
 * stepping.  Combines with any set of the switches above. */
#define SDE_FP64 128u
/* Variant of the method: the large-angle elastic cut (the upper limit
 * cos(2.5 sigma(E)) of Eq. (large_elastic_cm) and of the CM cosine drawn by
 * Eq. (large_elastic_cdf)) is 2.5 sigma(E), sigma the Lynch-Dahl width of
 * section 2.1.4 for the step's medium and density over the path ld_z_cm,
 * instead of the fixed theta_cut_rad the paper's runs use (the paper names
 * the energy-dependent cut, section 2.1.4, and leaves it for later,
 * section 4).  Limited to pi (pi - backscatter_cut_rad for hydrogen), where
 * the elastic rate vanishes.  Runs in the general instance. */
#define SDE_ECUT 256u

/* Ledger slots (sde_transport_ex ledger_out) */
#define SDE_LEDGER_DEPOSITED 0   /* energy scored inside the phantom (fixed point) */
#define SDE_LEDGER_ESCAPED 1     /* energy carried or scored outside (fixed point) */
#define SDE_LEDGER_NUCLEAR 2     /* energy removed by inelastic jumps (fixed point) */
#define SDE_LEDGER_INITIAL 3     /* source energy (fixed point) */
#define SDE_LEDGER_TRUNCATED 4   /* energy of histories stopped at max_steps */
#define SDE_LEDGER_STEPS 5       /* number of steps (count) */
#define SDE_LEDGER_HISTORIES 6   /* number of histories (count) */
#define SDE_LEDGER_JUMPS 7       /* number of large-angle jumps (count) */
#define SDE_LEDGER_BAD_LANES 8   /* energy of histories ended by the lane guard: a non-finite
                                    energy or direction (fixed point; 0 in a sound run) */
#define SDE_LEDGER_N 9

/* A medium: element list with mass fractions and one mean excitation
 * energy (section 2.1.3, Bragg additivity).  (host) */
typedef struct {
    int n_elem;            /* 1..SDE_MAX_ELEM */
    const int* Z;          /* atomic numbers */
    const double* A;       /* atomic weights, g/mol */
    const double* w;       /* mass fractions (renormalised to sum 1) */
    double I_eV;           /* mean excitation energy */
} sde_material_desc;

/* Scheme parameters; the paper's run values are step 0.05 cm, z 0.05 cm,
 * e_min 0.05 MeV, F 0.98, cuts 0.02 and 0.04 rad (sections 2.1, 2.2.2). */
typedef struct {
    double step_cm;              /* Delta, the track-length step */
    double ld_z_cm;              /* path length z of the Lynch-Dahl width */
    double e_min_MeV;            /* absorption energy; lower end of the tables */
    double e_max_MeV;            /* upper end of the tables */
    double ld_F;                 /* Lynch-Dahl central fraction */
    double theta_cut_rad;        /* large-angle elastic cut (CM) */
    double backscatter_cut_rad;  /* hydrogen backscatter cut (CM) */
    int n_energy;                /* lattice points, uniform in ln E (>= 16) */
    unsigned flags;              /* SDE_* physics switches */
    int64_t max_steps;           /* histories still alive after this many steps stop */
} sde_physics_params;

/* Nuclear data on the energy lattice of the physics params (n_energy
 * points uniform in ln E over [e_min, e_max]).  (host)
 *
 * Inelastic proton-nucleus interactions (section 2.1.5); values between
 * lattice points are linear in the lattice coordinate.  sigma_barn[t][i]
 * total cross section of element Z[t] at E_i (barn); u_icdf[t][i][j] inverse
 * CDF of the loss fraction u at U = j/(n_u-1); kalbach_r/kalbach_a[t][i][j]
 * Kalbach-Mann r and a at u = j/(n_u-1).
 *
 * Elastic nuclear terms (section 2.1.4), optional (counts 0 = none):
 *  - elements other than hydrogen, the nuclear-plus-interference term
 *    sigma_NI(E) P_NI(mu, E) of Eq. (elastic_large_barns): ni_sigma_barn[t][i]
 *    (barn) and ni_p[t][i][j], the cubic B-spline coefficients of
 *    P_NI(mu, E_i) (barn/sr per barn) on uniform knots over mu in [-1, 1]
 *    (knot j at -1 + (j - 3) 2/(n_mu - 3); n_mu in 7..256); the term is
 *    linear in the lattice coordinate between lattice energies;
 *  - hydrogen, the nuclear term of Eq. (hydrogen_not_ruther) for
 *    l = 0..n_l-1 (n_l <= 8): h_a_re, h_a_im, h_b [l][n_energy + 2], the
 *    cubic B-spline coefficients in the lattice coordinate (uniform knots at
 *    the lattice points, knot k at k - 3) of Re a_l(E), Im a_l(E) and b_l(E)
 *    (barn).
 *  The summed cross sections must be positive over the sampled range.
 * Refused with SDE_E_INVALID: negative or non-finite cross sections; an
 * inverse CDF outside [0, 1] or decreasing in U; Kalbach r outside [0, 1]
 * or a negative; non-finite B-spline coefficients; counts out of range. */
typedef struct {
    int n_tab;
    int n_u;                     /* >= 2 */
    const int* Z;                /* [n_tab] */
    const double* sigma_barn;    /* [n_tab][n_energy] */
    const double* u_icdf;        /* [n_tab][n_energy][n_u] */
    const double* kalbach_r;     /* [n_tab][n_energy][n_u] */
    const double* kalbach_a;     /* [n_tab][n_energy][n_u] */
    int n_ni;                    /* elements with sigma_NI P_NI (Z > 1), <= 64 */
    int n_mu;
    const int* ni_Z;             /* [n_ni] */
    const double* ni_sigma_barn; /* [n_ni][n_energy] */
    const double* ni_p;          /* [n_ni][n_energy][n_mu] */
    int n_l;                     /* hydrogen partial waves, 0..8 */
    const double* h_a_re;        /* [n_l][n_energy + 2] */
    const double* h_a_im;
    const double* h_b;
} sde_nuclear_tables;

/* Gaussian pencil beam along +z starting on the entrance face.  Each of its
 * n_histories histories carries weight / n_histories.  (host) */
typedef struct {
    double E_MeV;          /* nominal energy */
    double sigmaE_rel;     /* relative Gaussian energy spread */
    double x_cm, y_cm;     /* lateral centre */
    double sigma_xy_cm;    /* lateral Gaussian spread */
    double weight;         /* protons represented by the spot */
    uint64_t n_histories;
} sde_spot;

typedef struct {
    int n_spots;
    const sde_spot* spots; /* (host) [n_spots] */
} sde_beam;

/* Voxel phantom; D is the closed box [origin, origin + n d].  (device) */
typedef struct {
    int nx, ny, nz;
    double dx_cm, dy_cm, dz_cm;
    double origin_cm[3];            /* low corner */
    const uint8_t* material_id;     /* (device) [nz][ny][nx], < n_mats */
    const float* density;           /* (device) [nz][ny][nx], g/cm^3, > 0 */
} sde_phantom;

/* Launch configuration; zero fields take defaults.  Results do not depend
 * on it. */
typedef struct {
    int block;        /* threads per workgroup, multiple of 64, <= 1024 (512) */
    int grid;         /* workgroups (0: 2 per compute unit) */
    int refill;       /* refill when at least this many lanes of a wave are idle, 1..64 (8) */
    int jump_batch;   /* finish deferred jumps when this many lanes of a wave wait, 1..64 (8) */
    int tally_replicas; /* global tally copies, chosen per XCD and summed at the end, 1..16 (8) */
    int claim_chunk;  /* history indices a wave takes from the work counter at once, >= 64 (64) */
    int tile_nx, tile_ny, tile_nz;   /* LDS tally tile extent in voxels (0: none) */
    int tile_x0, tile_y0, tile_z0;   /* tile low corner in voxels */
    uint64_t nan_history;  /* test hook: 0 none; else history nan_history - 1 starts with a
                              NaN direction, which the lane guard must catch */
} sde_launch;

/* Build the per-material tables (FP64 on the host, FP32 hot fields staged in
 * LDS by the kernel, FP64 residual range) and upload them.  nuclear may be
 * NULL: then no element has an inelastic channel.  Replaces earlier tables.
 * Errors: SDE_E_INVALID (counts, fractions, I, lattice, a medium whose
 * stopping power is not positive at e_min), SDE_E_HIP, SDE_E_NOMEM. */
int sde_init_materials(const sde_material_desc* mats, int n_mats,
                       const sde_physics_params* params,
                       const sde_nuclear_tables* nuclear);

/* Stream for subsequent work (a hipStream_t; NULL = null stream). */
int sde_set_stream(void* hip_stream);

/* Transport the beam through the phantom and write dose-to-medium (Gy) for
 * the protons the spots represent into dose_out (device, nx*ny*nz doubles).
 * n_histories: 0 = the spots' counts; for a single spot a non-zero value
 * replaces its count; otherwise it must equal the sum of the counts.
 * Errors: SDE_E_STATE, SDE_E_INVALID, SDE_E_RANGE (a spot energy, with its
 * 5.77 sigma spread, outside the tables), SDE_E_OVERFLOW, SDE_E_HIP. */
int sde_transport(const sde_beam* beam, const sde_phantom* phantom, uint64_t n_histories,
                  uint64_t seed, double* dose_out);

/* As sde_transport, and also: tally_out (device, nvox int64, may be NULL)
 * receives the fixed-point tally (energy x scale, MeV); ledger_out (host,
 * SDE_LEDGER_N int64, may be NULL) the energy balance; scale_out (host, may
 * be NULL) the scale (2^k per MeV); launch (may be NULL) the configuration. */
int sde_transport_ex(const sde_beam* beam, const sde_phantom* phantom, uint64_t n_histories,
                     uint64_t seed, double* dose_out, int64_t* tally_out, int64_t* ledger_out,
                     double* scale_out, const sde_launch* launch);

/* Plans: a beam + phantom + seed prepared once (spot table, fixed-point
 * scale, packed voxel data uploaded), then executed as one persistent
 * launch; sde_plan_execute records the reset/transport/convert sequence in a
 * hipGraph on first use and replays it afterwards.  dose_out (device) may
 * change between calls (the graph is re-recorded).  The plan keeps its own
 * packed copy of the phantom, so the caller's voxel arrays may be freed after
 * sde_plan_create returns.  use_graph: 0 = plain launches, 1 = hipGraph. */
typedef struct sde_plan sde_plan;
int sde_plan_create(const sde_beam* beam, const sde_phantom* phantom, uint64_t n_histories,
                    uint64_t seed, const sde_launch* launch, sde_plan** plan_out);
int sde_plan_execute(sde_plan* plan, double* dose_out, int use_graph);
/* Results of the last execution: tally_out (device, nvox int64, may be NULL)
 * receives a copy of the fixed-point tally, ledger_out (host, SDE_LEDGER_N,
 * may be NULL) the ledger, scale_out (host, may be NULL) the scale.
 * Synchronises the stream. */
int sde_plan_results(sde_plan* plan, int64_t* tally_out, int64_t* ledger_out,
                     double* scale_out);
int sde_plan_destroy(sde_plan* plan);
/* Duration (ms) of the transport kernel of the last non-graph execution,
 * from HIP events recorded on the plan's stream around that launch.
 * Synchronises on the stop event.  SDE_E_STATE if none was recorded. */
int sde_plan_kernel_ms(sde_plan* plan, float* ms_out);
/* Optional per-history records for diagnosis: rec (device, n_histories x 12
 * floats, NULL = off) receives {E0, steps, jumps, end, x, y, z, E, first
 * jump step, last jump step, 0, 0} when a history ends, end being 1 end of
 * range, 2 left the phantom, 3 below e_min, 4 step limit, 5 started outside
 * or below e_min; (x, y, z) is where it stopped and E its energy at that
 * event (-1 jump steps: none).  Applies to later executions. */
int sde_plan_set_records(sde_plan* plan, float* rec);

/* Gamma index pass count (section 2.2.3): for each reference voxel with
 * dose >= thresh * max(ref), gamma = min over offsets x on the lattice of
 * spacing dta/interp within distance dta of
 * sqrt(|x|^2/dta^2 + (De(r+x) - Dr)^2 / (dd * norm)^2), De trilinear in the
 * evaluated grid (offsets leaving the grid are skipped), norm = Dr if local
 * else max(ref).  ref, eval: (device) [nz][ny][nx] doubles.
 * counts_out (host, 2): voxels evaluated, voxels with gamma <= 1. */
int sde_gamma(const double* ref, const double* eval, int nx, int ny, int nz, double dx_cm,
              double dy_cm, double dz_cm, double dd, double dta_cm, double thresh,
              int interp, int local, int64_t* counts_out);

/* sde_gamma for callers that cannot allocate device memory (code under
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same counts, with the counters and the search list in a
 * fixed scratch array of 4 MiB + 256 bytes that every GPU the library runs on
 * holds until the process ends; it calls no hipMalloc or hipFree.  Voxels
 * failing at the zero offset beyond 2^20 are searched in the first pass
 * (same counts, slower).  Calls on one GPU share its scratch array: calls
 * that overlap on one GPU (several host threads or streams) race.
 * Arguments, synchronisation and errors as sde_gamma; also SDE_E_INVALID for
 * more than 2^31 voxels. */
int sde_gamma_noalloc(const double* ref, const double* eval, int nx, int ny, int nz,
                      double dx_cm, double dy_cm, double dz_cm, double dd, double dta_cm,
                      double thresh, int interp, int local, int64_t* counts_out);

/* Kernel test entry point: the polar angle of the small-angle step as the
 * transport draws it with SDE_SBM (section 2.2.2; spherical Brownian motion
 * on S^2 at time t[i]: for t < 0.02 Algorithm 1 of Mijatovic et al. with
 * the lineage count Griffiths' normal rounded, mean + sd * z[i], and
 * X ~ Beta(1, 1 + M) by inversion of u[i]; else the exact inversion
 * P(cos <= c) = u[i] of the heat kernel's Legendre series).  t, u, z,
 * cos_out, sin_out: (device) float arrays of n; u in (0, 1), t >= 0.
 * Synchronises the stream.  SDE_E_INVALID for n < 0, n > 2^30 or a NULL
 * pointer with n > 0. */
int sde_sbm_polar(const float* t, const float* u, const float* z, int64_t n, float* cos_out,
                  float* sin_out);

/* Kernel test entry point: the transport's random numbers.  For i < count,
 * words_out[4i..4i+3] (device, 16-byte aligned) receives the Philox4x32-10
 * block (Salmon et al., SC'11; ten rounds) with key (seed low, seed high)
 * and counter (h[i] low, h[i] high, n[i], b[i]), the stream the transport
 * reads for history h, step n and block b (the source uses n = 2^32 - 1).
 * h, n, b: (device) arrays of count.  Synchronises the stream.
 * SDE_E_INVALID for count < 0, count > 2^30, a NULL or misaligned array
 * with count > 0. */
int sde_philox_words(uint64_t seed, const uint64_t* h, const uint32_t* n, const uint32_t* b,
                     int64_t count, uint32_t* words_out);

/* Launch limits for choosing a configuration: compute units, LDS bytes per
 * workgroup, and LDS bytes the current tables take (0 before
 * sde_init_materials).  Any pointer may be NULL. */
int sde_launch_limits(int* n_cu, int* max_lds_bytes, int* table_lds_bytes);

/* Release tables, buffers and plans-independent state. */
void sde_free(void);

/* Message of the last error on this thread ("" if none). */
const char* sde_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SDE_H */

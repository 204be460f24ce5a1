// C ABI of libsde (declared in include/sde.h): validation, device tables,
// plans (persistent launch + hipGraph replay), dose conversion and gamma.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "sde.h"
#include "sde_host.hpp"
#include "sde_internal.hpp"
#include "nn_internal.hpp"

using namespace sde;

namespace {

thread_local std::string g_err;

struct State {
    bool ready = false;
    HostTables host;
    float4* hot = nullptr;
    double2* rg64 = nullptr;
    MatDev* mats = nullptr;
    float *nuc_sigma = nullptr, *nuc_u = nullptr, *nuc_r = nullptr, *nuc_a = nullptr;
    MatDev64* mats64 = nullptr;
    double2* hot64 = nullptr;
    double *nuc_sigma64 = nullptr, *nuc_u64 = nullptr, *nuc_r64 = nullptr, *nuc_a64 = nullptr;
    float *ni_p = nullptr, *ni_cum = nullptr, *ni_sig = nullptr;
    double *ni_p64 = nullptr, *ni_cum64 = nullptr, *ni_sig64 = nullptr, *h_coef = nullptr;
    // gamma: the counters and the list of voxels to search
    unsigned long long* gam_buf = nullptr;
    unsigned* gam_list = nullptr;
    unsigned gam_cap = 0;
    hipStream_t stream = nullptr;
    hipStream_t own = nullptr;   // for graph capture when the caller uses the null stream
    int n_cu = 0;
    size_t max_lds = 0;
};
State g;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? SDE_E_NOMEM : SDE_E_HIP,              \
                        std::string(#expr) + ": " + hipGetErrorString(e_));               \
    } while (0)

template <class T>
void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

void release_tables() {
    dfree(g.hot);
    dfree(g.rg64);
    dfree(g.mats);
    dfree(g.nuc_sigma);
    dfree(g.nuc_u);
    dfree(g.nuc_r);
    dfree(g.nuc_a);
    dfree(g.mats64);
    dfree(g.hot64);
    dfree(g.nuc_sigma64);
    dfree(g.nuc_u64);
    dfree(g.nuc_r64);
    dfree(g.nuc_a64);
    dfree(g.ni_p);
    dfree(g.ni_cum);
    dfree(g.ni_sig);
    dfree(g.ni_p64);
    dfree(g.ni_cum64);
    dfree(g.ni_sig64);
    dfree(g.h_coef);
    g.ready = false;
}

template <class T>
int upload(T** dst, const std::vector<T>& src) {
    HIP_TRY(hipMalloc((void**)dst, sizeof(T) * std::max<size_t>(src.size(), 1)));
    HIP_TRY(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return SDE_OK;
}

int device_info() {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int cu = 0, lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    g.n_cu = cu;
    g.max_lds = (size_t)lds;
    HIP_TRY(transport_kernel_attributes(g.max_lds));
    return SDE_OK;
}

hipStream_t cur_stream() { return g.stream; }

}  // namespace

namespace sde {
hipStream_t library_stream() { return g.stream; }
int report_error(int code, const char* msg) { return fail(code, msg); }
}  // namespace sde

struct sde_plan {
    KParams kp{};
    int grid = 0, block = 0;
    size_t lds = 0;
    uint2* vox = nullptr;
    unsigned long long* tally = nullptr;
    unsigned long long* ledger = nullptr;
    unsigned long long* counter = nullptr;
    unsigned int* bad = nullptr;    // [1 + kMaxMat]: invalid-voxel count, per-material max density
    SpotDev* spots = nullptr;
    SpotDev64* spots64 = nullptr;
    unsigned long long* prefix = nullptr;
    size_t nvox = 0;
    int n_rep = 1;
    double scale = 1.0;
    double voxel_cm3 = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    double* graph_dose = nullptr;
    hipStream_t graph_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
};

namespace {

void plan_free(sde_plan* p) {
    if (!p) return;
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    dfree(p->vox);
    dfree(p->tally);
    dfree(p->ledger);
    dfree(p->counter);
    dfree(p->bad);
    dfree(p->spots);
    dfree(p->spots64);
    dfree(p->prefix);
    delete p;
}

// Enqueue reset, transport and the replica sum / dose conversion on stream s
// (dose_out may be NULL); with timing, HIP events bracket the transport launch.
int plan_enqueue(sde_plan* p, double* dose_out, hipStream_t s, bool timing = false) {
    HIP_TRY(launch_reset(p->tally, p->nvox * p->n_rep, p->ledger, p->counter, s));
    if (timing) {
        if (!p->ev0) HIP_TRY(hipEventCreate(&p->ev0));
        if (!p->ev1) HIP_TRY(hipEventCreate(&p->ev1));
        HIP_TRY(hipEventRecord(p->ev0, s));
    }
    HIP_TRY(launch_transport(p->kp, p->grid, p->block, p->lds, s));
    if (timing) {
        HIP_TRY(hipEventRecord(p->ev1, s));
        p->timed = true;
    }
    HIP_TRY(launch_convert(p->tally, p->n_rep, p->vox, p->nvox, 1.0 / p->scale, p->voxel_cm3,
                           dose_out, p->ledger, s));
    return SDE_OK;
}

int make_plan(const sde_beam* beam, const sde_phantom* ph, uint64_t n_histories, uint64_t seed,
              const sde_launch* launch, sde_plan** out) {
    if (!g.ready) return fail(SDE_E_STATE, "sde_init_materials has not been called");
    if (!beam || beam->n_spots < 1 || !beam->spots) return fail(SDE_E_INVALID, "empty beam");
    if (!ph || ph->nx < 1 || ph->ny < 1 || ph->nz < 1 || !(ph->dx_cm > 0) || !(ph->dy_cm > 0) ||
        !(ph->dz_cm > 0) || !ph->material_id || !ph->density)
        return fail(SDE_E_INVALID, "invalid phantom");
    const size_t nvox = (size_t)ph->nx * ph->ny * ph->nz;
    if (nvox >= (1ull << 31)) return fail(SDE_E_INVALID, "phantom too large (>= 2^31 voxels)");
    const HostTables& T = g.host;
    const sde_physics_params& pp = T.params;

    // history counts
    const int ns = beam->n_spots;
    std::vector<uint64_t> counts(ns);
    uint64_t total = 0;
    for (int i = 0; i < ns; ++i) {
        counts[i] = beam->spots[i].n_histories;
        total += counts[i];
    }
    if (n_histories) {
        if (ns == 1) {
            counts[0] = n_histories;
            total = n_histories;
        } else if (n_histories != total) {
            return fail(SDE_E_INVALID, "n_histories differs from the sum of the spot counts");
        }
    }
    if (total == 0) return fail(SDE_E_INVALID, "no histories");

    // energy range and fixed-point scale
    double emax_sum = 0;
    for (int i = 0; i < ns; ++i) {
        const sde_spot& s = beam->spots[i];
        if (!(s.E_MeV > 0) || !(s.sigmaE_rel >= 0) || !(s.sigma_xy_cm >= 0) || !(s.weight >= 0) ||
            !std::isfinite(s.x_cm) || !std::isfinite(s.y_cm))
            return fail(SDE_E_INVALID, "invalid spot " + std::to_string(i));
        if (counts[i] == 0) continue;
        const double ehi = s.E_MeV * (1.0 + kBoxMullerMax * s.sigmaE_rel);
        if (ehi > pp.e_max_MeV)
            return fail(SDE_E_RANGE, "spot " + std::to_string(i) + " energy exceeds e_max");
        if (s.E_MeV * (1.0 - kBoxMullerMax * s.sigmaE_rel) < 0.0)
            return fail(SDE_E_RANGE, "spot " + std::to_string(i) + " energy spread reaches zero");
        emax_sum += s.weight * ehi;
    }
    if (!(emax_sum > 0) || !std::isfinite(emax_sum))
        return fail(SDE_E_INVALID, "total weighted energy must be positive and finite");
    const int k = (int)std::floor(62.0 - std::log2(emax_sum));
    if (k < -60 || k > 100) return fail(SDE_E_OVERFLOW, "fixed-point scale out of range");
    const double scale = std::ldexp(1.0, k);

    sde_launch L{};
    if (launch) L = *launch;
    const int n_rep = L.tally_replicas ? L.tally_replicas : 8;
    if (n_rep < 1 || n_rep > 16) return fail(SDE_E_INVALID, "tally_replicas must be in 1..16");

    sde_plan* p = new sde_plan();
    p->nvox = nvox;
    p->n_rep = n_rep;
    p->scale = scale;
    p->voxel_cm3 = ph->dx_cm * ph->dy_cm * ph->dz_cm;

    // The kernel claims the spots' histories highest energy first (the
    // longest histories), so the last histories of a launch are short ones
    // and the lanes run out of work together.  Every history keeps its index
    // in the caller's spot order (h0 + offset), which keys its random
    // numbers: the result does not depend on this order.
    std::vector<unsigned long long> h0(ns + 1, 0);
    for (int i = 0; i < ns; ++i) h0[i + 1] = h0[i] + counts[i];
    std::vector<int> order(ns);
    for (int i = 0; i < ns; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return beam->spots[a].E_MeV > beam->spots[b].E_MeV;
    });
    std::vector<SpotDev> sd(ns);
    std::vector<SpotDev64> sd64(ns);
    std::vector<unsigned long long> pre(ns + 1, 0);   // prefix in claim order
    for (int k = 0; k < ns; ++k) {
        const int i = order[k];
        const sde_spot& s = beam->spots[i];
        const double wsc = counts[i] ? s.weight / (double)counts[i] * scale : 0.0;
        sd[k] = SpotDev{(float)s.E_MeV, (float)s.sigmaE_rel, (float)s.x_cm, (float)s.y_cm,
                        (float)s.sigma_xy_cm, (float)wsc, h0[i]};
        sd64[k] = SpotDev64{s.E_MeV, s.sigmaE_rel, s.x_cm, s.y_cm, s.sigma_xy_cm, wsc, h0[i]};
        pre[k + 1] = pre[k] + counts[i];
    }
    auto bail = [&](int rc) {
        plan_free(p);
        return rc;
    };
    int rc;
    if ((rc = upload(&p->spots, sd)) != SDE_OK) return bail(rc);
    if ((rc = upload(&p->spots64, sd64)) != SDE_OK) return bail(rc);
    if ((rc = upload(&p->prefix, pre)) != SDE_OK) return bail(rc);
    hipError_t e;
    if ((e = hipMalloc((void**)&p->vox, sizeof(uint2) * nvox)) != hipSuccess ||
        (e = hipMalloc((void**)&p->tally, sizeof(unsigned long long) * nvox * n_rep)) != hipSuccess ||
        (e = hipMalloc((void**)&p->ledger, sizeof(unsigned long long) * kLedgerN)) != hipSuccess ||
        (e = hipMalloc((void**)&p->counter, sizeof(unsigned long long))) != hipSuccess ||
        (e = hipMalloc((void**)&p->bad, sizeof(unsigned int) * (1 + kMaxMat))) != hipSuccess) {
        plan_free(p);
        return fail(SDE_E_NOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    }
    hipStream_t s = cur_stream();
    if ((e = hipMemsetAsync(p->bad, 0, sizeof(unsigned int) * (1 + kMaxMat), s)) != hipSuccess ||
        (e = launch_pack_phantom(ph->material_id, ph->density, p->vox, nvox, T.n_mat, p->bad,
                                 p->bad + 1, s)) != hipSuccess) {
        plan_free(p);
        return fail(SDE_E_HIP, std::string("phantom packing failed: ") + hipGetErrorString(e));
    }
    unsigned int chk[1 + kMaxMat] = {0};
    if ((e = hipMemcpyAsync(chk, p->bad, sizeof chk, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
        plan_free(p);
        return fail(SDE_E_HIP, std::string("phantom check failed: ") + hipGetErrorString(e));
    }
    const unsigned int bad = chk[0];
    if (bad) {
        plan_free(p);
        return fail(SDE_E_INVALID, std::to_string(bad) +
                                       " voxels have a material id >= n_mats or a density that "
                                       "is not finite and positive");
    }

    // launch configuration
    int block = L.block ? L.block : 512;
    if (block < 64 || block > 1024 || block % 64) {
        plan_free(p);
        return fail(SDE_E_INVALID, "block must be a multiple of 64 in 64..1024");
    }
    int grid = L.grid ? L.grid : 2 * std::max(1, g.n_cu);
    if (grid < 1) grid = 1;
    int refill = L.refill ? L.refill : 8;
    if (refill < 1 || refill > 64) {
        plan_free(p);
        return fail(SDE_E_INVALID, "refill must be in 1..64");
    }
    const int claim_chunk = L.claim_chunk ? L.claim_chunk : 64;
    if (claim_chunk < 64 || claim_chunk > (1 << 20)) {
        plan_free(p);
        return fail(SDE_E_INVALID, "claim_chunk must be in 64..2^20");
    }
    int jump_batch = L.jump_batch ? L.jump_batch : 8;
    if (jump_batch < 1 || jump_batch > 64) {
        plan_free(p);
        return fail(SDE_E_INVALID, "jump_batch must be in 1..64");
    }
    const int tnx = std::max(0, L.tile_nx), tny = std::max(0, L.tile_ny),
              tnz = std::max(0, L.tile_nz);
    const bool tile_on = tnx > 0 && tny > 0 && tnz > 0;
    if (tile_on && (L.tile_x0 < 0 || L.tile_y0 < 0 || L.tile_z0 < 0 ||
                    L.tile_x0 + tnx > ph->nx || L.tile_y0 + tny > ph->ny ||
                    L.tile_z0 + tnz > ph->nz)) {
        plan_free(p);
        return fail(SDE_E_INVALID, "LDS tile outside the phantom");
    }
    const size_t tab_bytes = ((size_t)T.n_mat * T.n_e + T.n_mat) * sizeof(float4);
    const size_t tile_bytes = tile_on ? (size_t)tnx * tny * tnz * 8 : 0;
    if (tab_bytes + tile_bytes > g.max_lds) {
        plan_free(p);
        return fail(SDE_E_INVALID, "tables and tally tile exceed the LDS per workgroup (" +
                                       std::to_string(tab_bytes + tile_bytes) + " > " +
                                       std::to_string(g.max_lds) + " bytes)");
    }
    p->grid = grid;
    p->block = block;
    p->lds = tab_bytes + tile_bytes;

    KParams& kp = p->kp;
    kp.hot = g.hot;
    kp.rg64 = g.rg64;
    kp.mats = g.mats;
    kp.nuc_sigma = g.nuc_sigma;
    kp.nuc_u = g.nuc_u;
    kp.nuc_r = g.nuc_r;
    kp.nuc_a = g.nuc_a;
    kp.n_mat = T.n_mat;
    kp.n_e = T.n_e;
    kp.n_u = T.n_u;
    kp.n_tab = T.n_tab;
    kp.mats64 = g.mats64;
    kp.hot64 = g.hot64;
    kp.nuc_sigma64 = g.nuc_sigma64;
    kp.nuc_u64 = g.nuc_u64;
    kp.nuc_r64 = g.nuc_r64;
    kp.nuc_a64 = g.nuc_a64;
    kp.n_ni = T.n_ni;
    kp.n_mu = T.n_mu;
    kp.n_l = T.n_l;
    kp.ni_p = g.ni_p;
    kp.ni_cum = g.ni_cum;
    kp.ni_sig = g.ni_sig;
    kp.ni_p64 = g.ni_p64;
    kp.ni_cum64 = g.ni_cum64;
    kp.ni_sig64 = g.ni_sig64;
    kp.h_coef = g.h_coef;
    // scheme and geometry scalars, in double and rounded to float
    KScal<double>& S = kp.sd;
    S.step = pp.step_cm;
    S.half_step = 0.5 * pp.step_cm;
    S.sqrt_step = std::sqrt(pp.step_cm);
    S.e_min = pp.e_min_MeV;
    S.c_bethe = kBethe;
    S.c_strag = T.c_strag;
    S.ruth_T = T.ruth_T;
    S.mott_lo = T.mott_lo;
    S.mott_hi = T.mott_hi;
    S.mott_D0 = T.mott_D0;
    S.mott_Lhi = T.mott_Lhi;
    S.mott_Llo = T.mott_Llo;
    S.mott_Dlo = T.mott_Dlo;
    S.mott_shi = T.mott_shi;
    S.mott_slo = T.mott_slo;
    S.z_over_step = pp.ld_z_cm / pp.step_cm;
    S.eta_pre = kAlpha * std::sqrt(0.5 * kMp);
    S.ln_e_lo = T.ln_e_lo;
    S.inv_dln = 1.0 / T.dln;
    S.ld_z = pp.ld_z_cm;
    S.ld_F = pp.ld_F;
    const double d[3] = {ph->dx_cm, ph->dy_cm, ph->dz_cm};
    const int nn[3] = {ph->nx, ph->ny, ph->nz};
    for (int a = 0; a < 3; ++a) {
        S.lo[a] = ph->origin_cm[a];
        S.hi[a] = ph->origin_cm[a] + nn[a] * d[a];
        S.d[a] = d[a];
        S.inv_d[a] = 1.0 / d[a];
    }
    KScal<float>& F = kp.sf;
    F.step = (float)S.step;
    F.half_step = (float)S.half_step;
    F.sqrt_step = (float)S.sqrt_step;
    F.e_min = (float)S.e_min;
    F.c_bethe = (float)S.c_bethe;
    F.c_strag = (float)S.c_strag;
    F.ruth_T = (float)S.ruth_T;
    F.mott_lo = (float)S.mott_lo;
    F.mott_hi = (float)S.mott_hi;
    F.mott_D0 = (float)S.mott_D0;
    F.mott_Lhi = (float)S.mott_Lhi;
    F.mott_Llo = (float)S.mott_Llo;
    F.mott_Dlo = (float)S.mott_Dlo;
    F.mott_shi = (float)S.mott_shi;
    F.mott_slo = (float)S.mott_slo;
    F.z_over_step = (float)S.z_over_step;
    F.eta_pre = (float)S.eta_pre;
    F.ln_e_lo = (float)S.ln_e_lo;
    F.inv_dln = (float)S.inv_dln;
    F.ld_z = (float)S.ld_z;
    F.ld_F = (float)S.ld_F;
    for (int a = 0; a < 3; ++a) {
        F.lo[a] = (float)S.lo[a];
        F.hi[a] = (float)S.hi[a];
        F.d[a] = (float)S.d[a];
        F.inv_d[a] = (float)S.inv_d[a];
    }
    kp.flags = pp.flags & (SDE_ALL | SDE_ECUT);
    kp.fp64 = (pp.flags & SDE_FP64) ? 1 : 0;
    kp.max_steps = pp.max_steps;
    kp.vox = p->vox;
    kp.nx = ph->nx;
    kp.ny = ph->ny;
    kp.nz = ph->nz;
    kp.spots = p->spots;
    kp.spots64 = p->spots64;
    kp.prefix = p->prefix;
    kp.n_spots = ns;
    kp.n_hist = total;
    kp.seed = seed;
    kp.tally = p->tally;
    kp.rep_stride = nvox;
    kp.n_rep = n_rep;
    kp.ledger = p->ledger;
    kp.counter = p->counter;
    kp.refill = refill;
    kp.jump_batch = jump_batch;
    kp.nan_h = L.nan_history ? L.nan_history - 1 : ~0ull;
    kp.claim_chunk = claim_chunk;
    // End-of-range screen: for E above ec[m] the residual range exceeds the
    // step at every voxel of material m (densest voxel, 0.1 % margin); below
    // it the kernel decides in FP64.
    for (int m = 0; m < kMaxMat; ++m) kp.ec[m] = 0.0f;
    for (int m = 0; m < T.n_mat; ++m) {
        float rmax;
        std::memcpy(&rmax, &chk[1 + m], sizeof rmax);
        if (!(rmax > 0.0f)) continue;
        const double limit = pp.step_cm * (double)rmax * 1.001;
        double ec = T.e_hi;
        for (int j = 0; j < T.n_e; ++j)
            if (T.rg64[(size_t)m * T.n_e + j].x >= limit) {
                ec = std::exp(T.ln_e_lo + j * T.dln);
                break;
            }
        kp.ec[m] = (float)(ec * (1.0 + 1e-6));
    }
    if (tile_on) {
        kp.tile_nx = tnx;
        kp.tile_ny = tny;
        kp.tile_nz = tnz;
        kp.tile_x0 = L.tile_x0;
        kp.tile_y0 = L.tile_y0;
        kp.tile_z0 = L.tile_z0;
    }
    *out = p;
    return SDE_OK;
}

// Gamma index: argument checks and the launch sequence.
int gamma_check(const double* ref, const double* ev, int nx, int ny, int nz, double dx_cm,
                double dy_cm, double dz_cm, double dd, double dta_cm, double thresh, int interp,
                const int64_t* counts_out) {
    if (!ref || !ev || !counts_out || nx < 1 || ny < 1 || nz < 1 || !(dx_cm > 0) ||
        !(dy_cm > 0) || !(dz_cm > 0) || !(dd > 0) || !(dta_cm > 0) || !(thresh >= 0) ||
        interp < 1 || interp > 50 || (double)nx * ny * nz >= 9.0e15)
        return fail(SDE_E_INVALID, "invalid gamma arguments");
    return SDE_OK;
}

// Counters and maximum into buf[0..3], then the two gamma passes with a
// search list of cap voxel indices; reads the counts back (synchronises the
// stream).
int gamma_run(const double* ref, const double* ev, int nx, int ny, int nz, double dx_cm,
              double dy_cm, double dz_cm, double dd, double dta_cm, double thresh, int interp,
              int local, unsigned long long* buf, unsigned* list, unsigned cap,
              int64_t* counts_out) {
    const size_t nvox = (size_t)nx * ny * nz;
    hipStream_t s = cur_stream();
    unsigned long long host[3] = {0, 0, 0};
    hipError_t e;
    if ((e = launch_zero_u64(buf, 4, s)) != hipSuccess ||
        (e = launch_max(ref, nvox, buf + 2, s)) != hipSuccess ||
        (e = hipMemcpyAsync(host, buf, sizeof host, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(SDE_E_HIP, hipGetErrorString(e));
    double mx;
    std::memcpy(&mx, &host[2], sizeof mx);
    // the per-octant cells and bounds need the search box inside the 8
    // cells around a voxel
    const int use_bound =
        (dta_cm / dx_cm < 1.0 && dta_cm / dy_cm < 1.0 && dta_cm / dz_cm < 1.0) ? 1 : 0;
    if ((e = launch_gamma(ref, ev, nx, ny, nz, interp, dta_cm, dx_cm, dy_cm, dz_cm, dd,
                          thresh * mx, mx, local, use_bound, buf, list, cap, s)) != hipSuccess ||
        (e = hipMemcpyAsync(host, buf, sizeof(unsigned long long) * 2, hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(SDE_E_HIP, hipGetErrorString(e));
    counts_out[0] = (int64_t)host[0];
    counts_out[1] = (int64_t)host[1];
    return SDE_OK;
}

// Scratch of sde_gamma_noalloc on each GPU: the four counters, then a
// search list of kNoallocList voxel indices (voxels beyond it are searched in
// the first pass).  In host code `scratch` is only a symbol: its device
// address comes from hipGetSymbolAddress, once per device.
constexpr unsigned kNoallocList = 1u << 20;
constexpr size_t kNoallocCounters = 256;   // bytes before the list
static __device__ __align__(256) unsigned char scratch[kNoallocCounters +
                                                       sizeof(unsigned) * kNoallocList];
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// This device's copy of the scratch array (its address looked up on the
// first call with that device current).
int noalloc_scratch(unsigned char** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SDE_E_INVALID, "device index out of range");
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = ptr;
    }
    *out = (unsigned char*)g_scratch_ptr[dev];
    return SDE_OK;
}

}  // namespace

extern "C" {

int sde_init_materials(const sde_material_desc* mats, int n_mats, const sde_physics_params* params,
                       const sde_nuclear_tables* nuclear) {
    g_err.clear();
    HostTables T;
    std::string err;
    const int rc = build_host_tables(mats, n_mats, params, nuclear, &T, &err);
    if (rc != SDE_OK) return fail(rc, err);
    release_tables();
    if (int r = device_info()) return r;
    int r;
    if ((r = upload(&g.hot, T.hot)) || (r = upload(&g.rg64, T.rg64)) ||
        (r = upload(&g.mats, T.mats)) || (r = upload(&g.nuc_sigma, T.nuc_sigma)) ||
        (r = upload(&g.nuc_u, T.nuc_u)) || (r = upload(&g.nuc_r, T.nuc_r)) ||
        (r = upload(&g.nuc_a, T.nuc_a)) || (r = upload(&g.mats64, T.mats64)) ||
        (r = upload(&g.hot64, T.hot64)) || (r = upload(&g.nuc_sigma64, T.nuc_sigma64)) ||
        (r = upload(&g.nuc_u64, T.nuc_u64)) || (r = upload(&g.nuc_r64, T.nuc_r64)) ||
        (r = upload(&g.nuc_a64, T.nuc_a64)) || (r = upload(&g.ni_p, T.ni_p)) ||
        (r = upload(&g.ni_cum, T.ni_cum)) || (r = upload(&g.ni_sig, T.ni_sig)) ||
        (r = upload(&g.ni_p64, T.ni_p64)) || (r = upload(&g.ni_cum64, T.ni_cum64)) ||
        (r = upload(&g.ni_sig64, T.ni_sig64)) || (r = upload(&g.h_coef, T.h_coef))) {
        release_tables();
        return r;
    }
    g.host = std::move(T);
    g.ready = true;
    return SDE_OK;
}

int sde_set_stream(void* hip_stream) {
    g.stream = (hipStream_t)hip_stream;
    return SDE_OK;
}

int sde_plan_create(const sde_beam* beam, const sde_phantom* phantom, uint64_t n_histories,
                    uint64_t seed, const sde_launch* launch, sde_plan** plan_out) {
    g_err.clear();
    if (!plan_out) return fail(SDE_E_INVALID, "plan_out is NULL");
    *plan_out = nullptr;
    return make_plan(beam, phantom, n_histories, seed, launch, plan_out);
}

int sde_plan_execute(sde_plan* p, double* dose_out, int use_graph) {
    g_err.clear();
    if (!p) return fail(SDE_E_INVALID, "plan is NULL");
    if (!use_graph) return plan_enqueue(p, dose_out, cur_stream(), true);
    hipStream_t s = cur_stream();
    if (!s) {
        if (!g.own) HIP_TRY(hipStreamCreate(&g.own));
        s = g.own;
    }
    if (!p->gexec || p->graph_dose != dose_out || p->graph_stream != s) {
        if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        p->gexec = nullptr;
        p->graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const int rc = plan_enqueue(p, dose_out, s);
        hipGraph_t gr = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &gr);
        if (rc != SDE_OK) {
            if (gr) (void)hipGraphDestroy(gr);
            return rc;
        }
        if (e != hipSuccess) return fail(SDE_E_HIP, std::string("capture: ") + hipGetErrorString(e));
        p->graph = gr;
        HIP_TRY(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
        p->graph_dose = dose_out;
        p->graph_stream = s;
    }
    HIP_TRY(hipGraphLaunch(p->gexec, s));
    if (s != cur_stream()) HIP_TRY(hipStreamSynchronize(s));
    return SDE_OK;
}

int sde_plan_results(sde_plan* p, int64_t* tally_out, int64_t* ledger_out, double* scale_out) {
    g_err.clear();
    if (!p) return fail(SDE_E_INVALID, "plan is NULL");
    if (scale_out) *scale_out = p->scale;
    hipStream_t s = cur_stream();
    if (p->graph_stream && p->graph_stream != s) HIP_TRY(hipStreamSynchronize(p->graph_stream));
    if (tally_out)
        HIP_TRY(hipMemcpyAsync(tally_out, p->tally, sizeof(int64_t) * p->nvox,
                               hipMemcpyDeviceToDevice, s));
    if (ledger_out)
        HIP_TRY(hipMemcpyAsync(ledger_out, p->ledger, sizeof(int64_t) * kLedgerN,
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SDE_OK;
}

int sde_plan_kernel_ms(sde_plan* p, float* ms_out) {
    g_err.clear();
    if (!p || !ms_out) return fail(SDE_E_INVALID, "plan or ms_out is NULL");
    if (!p->timed) return fail(SDE_E_STATE, "no timed execution");
    HIP_TRY(hipEventSynchronize(p->ev1));
    HIP_TRY(hipEventElapsedTime(ms_out, p->ev0, p->ev1));
    return SDE_OK;
}

int sde_plan_set_records(sde_plan* p, float* rec) {
    g_err.clear();
    if (!p) return fail(SDE_E_INVALID, "plan is NULL");
    p->kp.rec = rec;
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->gexec = nullptr;
    p->graph = nullptr;
    return SDE_OK;
}

int sde_plan_destroy(sde_plan* p) {
    g_err.clear();
    if (p) {
        (void)hipStreamSynchronize(cur_stream());
        plan_free(p);
    }
    return SDE_OK;
}

int sde_transport_ex(const sde_beam* beam, const sde_phantom* phantom, uint64_t n_histories,
                     uint64_t seed, double* dose_out, int64_t* tally_out, int64_t* ledger_out,
                     double* scale_out, const sde_launch* launch) {
    g_err.clear();
    sde_plan* p = nullptr;
    int rc = make_plan(beam, phantom, n_histories, seed, launch, &p);
    if (rc != SDE_OK) return rc;
    hipStream_t s = cur_stream();
    rc = plan_enqueue(p, dose_out, s);
    if (rc == SDE_OK && tally_out) {
        const hipError_t e = hipMemcpyAsync(tally_out, p->tally, sizeof(int64_t) * p->nvox,
                                            hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) rc = fail(SDE_E_HIP, hipGetErrorString(e));
    }
    if (rc == SDE_OK && ledger_out) {
        const hipError_t e = hipMemcpyAsync(ledger_out, p->ledger, sizeof(int64_t) * kLedgerN,
                                            hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) rc = fail(SDE_E_HIP, hipGetErrorString(e));
    }
    if (scale_out) *scale_out = p->scale;
    const hipError_t e = hipStreamSynchronize(s);
    if (rc == SDE_OK && e != hipSuccess) rc = fail(SDE_E_HIP, hipGetErrorString(e));
    plan_free(p);
    return rc;
}

int sde_transport(const sde_beam* beam, const sde_phantom* phantom, uint64_t n_histories,
                  uint64_t seed, double* dose_out) {
    if (!dose_out) return fail(SDE_E_INVALID, "dose_out is NULL");
    return sde_transport_ex(beam, phantom, n_histories, seed, dose_out, nullptr, nullptr, nullptr,
                            nullptr);
}

int sde_sbm_polar(const float* t, const float* u, const float* z, int64_t n, float* cos_out,
                  float* sin_out) {
    g_err.clear();
    if (n < 0 || n > (1ll << 30) || (n > 0 && (!t || !u || !z || !cos_out || !sin_out)))
        return fail(SDE_E_INVALID, "invalid sbm_polar arguments");
    if (n == 0) return SDE_OK;
    hipStream_t s = cur_stream();
    hipError_t e = launch_sbm_polar(t, u, z, (int)n, cos_out, sin_out, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? SDE_OK : fail(SDE_E_HIP, hipGetErrorString(e));
}

int sde_philox_words(uint64_t seed, const uint64_t* h, const uint32_t* n, const uint32_t* b,
                     int64_t count, uint32_t* words_out) {
    g_err.clear();
    if (count < 0 || count > (1ll << 30) || (count > 0 && (!h || !n || !b || !words_out)))
        return fail(SDE_E_INVALID, "invalid philox_words arguments");
    if ((uintptr_t)words_out % 16 != 0 || (uintptr_t)h % 8 != 0 || (uintptr_t)n % 4 != 0 ||
        (uintptr_t)b % 4 != 0)
        return fail(SDE_E_INVALID, "philox_words: misaligned array (words_out needs 16 bytes)");
    if (count == 0) return SDE_OK;
    hipStream_t s = cur_stream();
    hipError_t e = launch_philox_words(seed, (const unsigned long long*)h, n, b, (int)count,
                                       (uint4*)words_out, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? SDE_OK : fail(SDE_E_HIP, hipGetErrorString(e));
}

int sde_gamma(const double* ref, const double* ev, int nx, int ny, int nz, double dx_cm,
              double dy_cm, double dz_cm, double dd, double dta_cm, double thresh, int interp,
              int local, int64_t* counts_out) {
    g_err.clear();
    if (int rc = gamma_check(ref, ev, nx, ny, nz, dx_cm, dy_cm, dz_cm, dd, dta_cm, thresh, interp,
                             counts_out))
        return rc;
    // the counters and the search list, held by the library across calls
    // (the list grows to the largest grid seen, at most 2^24 entries;
    // beyond it voxels are searched in the first pass)
    if (!g.gam_buf) HIP_TRY(hipMalloc((void**)&g.gam_buf, sizeof(unsigned long long) * 4));
    const unsigned want = (unsigned)std::min<size_t>((size_t)nx * ny * nz, (size_t)1 << 24);
    if (want > g.gam_cap) {
        dfree(g.gam_list);
        g.gam_cap = 0;
        HIP_TRY(hipMalloc((void**)&g.gam_list, sizeof(unsigned) * want));
        g.gam_cap = want;
    }
    return gamma_run(ref, ev, nx, ny, nz, dx_cm, dy_cm, dz_cm, dd, dta_cm, thresh, interp, local,
                     g.gam_buf, g.gam_list, g.gam_cap, counts_out);
}

int sde_gamma_noalloc(const double* ref, const double* ev, int nx, int ny, int nz,
                      double dx_cm, double dy_cm, double dz_cm, double dd, double dta_cm,
                      double thresh, int interp, int local, int64_t* counts_out) {
    g_err.clear();
    if (int rc = gamma_check(ref, ev, nx, ny, nz, dx_cm, dy_cm, dz_cm, dd, dta_cm, thresh, interp,
                             counts_out))
        return rc;
    if ((size_t)nx * ny * nz > ((size_t)1 << 31))
        return fail(SDE_E_INVALID, "sde_gamma_noalloc: more than 2^31 voxels");
    unsigned char* sc = nullptr;
    if (int rc = noalloc_scratch(&sc)) return rc;
    return gamma_run(ref, ev, nx, ny, nz, dx_cm, dy_cm, dz_cm, dd, dta_cm, thresh, interp, local,
                     (unsigned long long*)sc, (unsigned*)(sc + kNoallocCounters), kNoallocList,
                     counts_out);
}

int sde_launch_limits(int* n_cu, int* max_lds_bytes, int* table_lds_bytes) {
    g_err.clear();
    if (!g.n_cu)
        if (int r = device_info()) return r;
    if (n_cu) *n_cu = g.n_cu;
    if (max_lds_bytes) *max_lds_bytes = (int)g.max_lds;
    if (table_lds_bytes)
        *table_lds_bytes = g.ready ? (int)(((size_t)g.host.n_mat * g.host.n_e + g.host.n_mat) *
                                           sizeof(float4))
                                   : 0;
    return SDE_OK;
}

void sde_free(void) {
    release_tables();
    dfree(g.gam_buf);
    dfree(g.gam_list);
    g.gam_cap = 0;
    if (g.own) {
        (void)hipStreamDestroy(g.own);
        g.own = nullptr;
    }
}

const char* sde_last_error(void) { return g_err.c_str(); }

}  // extern "C"

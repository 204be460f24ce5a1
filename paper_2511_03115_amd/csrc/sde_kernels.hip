// HIP kernels of libsde for gfx950 (CDNA4, wave64).
//
// k_transport: one lane per proton history in a persistent loop.  Lanes whose
// proton has stopped or left the phantom claim new history indices from a
// global counter, a wave at a time (one atomic per refill).  Each lane steps
// its history with the explicit Euler-Maruyama scheme of Eq. (VSDE):
// coefficients at Y_n, continuous loss with clamped straggling, small-angle
// diffusion, then a Poisson-clocked jump drawn from the mixture Eq. (Npi).
// Randomness is Philox4x32-10 keyed by the seed with counter
// (history, step, block), so a history's arithmetic does not depend on which
// lane, wave or launch runs it.  Energy is scored as int64 fixed point with
// integer atomics (an LDS tile first when one is configured), so the tally
// is the same for every launch shape.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sde_internal.hpp"

namespace sde {
namespace {

constexpr unsigned kLoss = 1u, kStraggle = 2u, kMcs = 4u, kElastic = 8u, kInelastic = 16u,
                   kEor = 32u, kSbm = 64u;
// the method (every switch) and the method with the geodesic Gaussian step:
// each its own compiled instance, the rest share k_transport<0> (switches
// read at run time)
constexpr unsigned kMethod = 127u, kMethodGeodesic = 63u;

constexpr float kMpF = (float)kMp;
constexpr float kLn2 = 0.69314718055994530942f;

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 32x32->64 products, key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
    // An empty barrier on the (wave-uniform) key: without it the compiler
    // hoists all twenty round keys out of the caller's loop, where they
    // occupy scalar registers for the whole kernel and are spilled; with it
    // they are rebuilt here by scalar adds.
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        // three-way xor in one gfx950 instruction (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// (2k+1) 2^-24 from the top 23 bits: exact in FP32, never 0 or 1.
__device__ __forceinline__ float u_hi(uint32_t w) { return ((float)(w >> 9) + 0.5f) * 0x1p-23f; }
// Same from the 23 low bits that u_hi leaves unused in three words.
__device__ __forceinline__ float u_lo(uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t k = (a & 0x1FFu) | ((b & 0x1FFu) << 9) | ((c & 0x1Fu) << 18);
    return ((float)k + 0.5f) * 0x1p-23f;
}

__device__ __forceinline__ float flog(float x) { return __builtin_amdgcn_logf(x) * kLn2; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// sin and cos of 2 pi u for u in (0, 1): the hardware takes revolutions.
__device__ __forceinline__ float sin_rev(float u) { return __builtin_amdgcn_sinf(u); }
__device__ __forceinline__ float cos_rev(float u) { return __builtin_amdgcn_cosf(u); }

// cos and sin of a polar angle given its square: Taylor in theta^2 for small
// angles (where the hardware sine would lose relative accuracy), the hardware
// sine and cosine (absolute error ~1e-7) otherwise.
__device__ __forceinline__ void polar_cs(float th2, float& c, float& s) {
    if (th2 < 0.25f) {
        const float x = th2;
        c = fmaf(x, fmaf(x, fmaf(x, fmaf(x, fmaf(x, -2.7557319e-7f, 2.4801587e-5f),
                                         -1.3888889e-3f), 4.1666667e-2f), -0.5f), 1.0f);
        const float sc = fmaf(x, fmaf(x, fmaf(x, fmaf(x, fmaf(x, -2.5052108e-8f, 2.7557319e-6f),
                                              -1.9841270e-4f), 8.3333333e-3f),
                                      -1.6666667e-1f), 1.0f);
        s = fsqrt(x) * sc;
    } else {
        const float r = sqrtf(th2) * 0.15915494309189535f;   // revolutions
        s = sin_rev(r);
        c = cos_rev(r);
    }
}

// Spherical Brownian motion on S^2 (generator half the Laplace-Beltrami
// operator) at time t = sigma^2 Delta / z, the law of the small-angle
// diffusion over one step (section 2.2.2), by the sampler the paper cites
// (Mijatovic, Mramor and Uribe Bravo 2020, Algorithm 1): M = the number of
// lineages left at time t of Kingman's coalescent with mutation parameter
// d - 1 = 2 started from infinitely many, X ~ Beta(1, 1 + M),
// cos = 1 - 2 X.  u -> 1 gives the angle -> 0 in both regimes.
constexpr float kSbmSwitch = 0.02f;
constexpr int kSbmL = 64;   // Legendre terms: e^{-l(l+1)t/2} < 1e-18 beyond, t >= kSbmSwitch

// t < kSbmSwitch: M from Griffiths' normal law, mean 2/t - 1/2 + t/24
// (series of 1/expm1(t/2), error t^3/5760) and standard deviation
// sqrt(2/(3t)) (1 - 7t^2/480), rounded to the nearest integer; then X by
// inversion, -expm1(ln u / (1 + M)) as a degree-7 polynomial: here
// 1 + M >= 67 (|z| <= 5.77) and -ln u <= 16.7, so |ln u / (1 + M)| <= 0.25
// and the truncation is below 2e-9 relative.
__device__ __forceinline__ void sbm_small(float t, float z, float u, float& ct, float& st) {
    t = fmaxf(t, 1e-30f);
    const float r = __builtin_amdgcn_rsqf(t);
    const float mu = fmaf(2.0f * r, r, fmaf(t, 1.0f / 24.0f, -0.5f));
    const float sd = 0.81649658f * r * fmaf(-7.0f / 480.0f * t, t, 1.0f);
    const float M = fmaxf(rintf(fmaf(sd, z, mu)), 0.0f);
    const float y = flog(u) * frcp(M + 1.0f);
    const float p = fmaf(y, fmaf(y, fmaf(y, fmaf(y, fmaf(y, fmaf(y, 1.0f / 5040.0f, 1.0f / 720.0f),
                                                         1.0f / 120.0f), 1.0f / 24.0f),
                                         1.0f / 6.0f), 0.5f), 1.0f);
    const float X = -y * p;
    ct = fmaf(-2.0f, X, 1.0f);
    st = 2.0f * fsqrt(X * (1.0f - X));
}

// Legendre recurrence coefficients (l+1) P_{l+1} = (2l+1) c P_l - l P_{l-1}
// as (2l+1)/(l+1) and l/(l+1), read with a wave-uniform index.
struct LegendreCoef {
    double a[kSbmL + 1], b[kSbmL + 1];
};
constexpr LegendreCoef legendre_coef() {
    LegendreCoef k{};
    for (int l = 0; l <= kSbmL; ++l) {
        k.a[l] = (2.0 * l + 1.0) / (l + 1.0);
        k.b[l] = (double)l / (l + 1.0);
    }
    return k;
}
__constant__ LegendreCoef kLegendre = legendre_coef();

// P(cos > c) at time t and its density in c, from the heat kernel on S^2,
// sum_l (2l+1)/2 e^{-l(l+1)t/2} P_l(c), whose integral from c to 1 has the
// terms (P_{l-1} - P_{l+1}) / 2 for l >= 1.  Weights by
// e^{-l(l+1)t/2} = e^{-(l-1)l t/2} (e^{-t})^l.  The loop stays rolled: its
// constants unrolled would crowd out the step's scalar registers.
__device__ __forceinline__ void sbm_tail(double q, double c, double& g, double& f) {
    double ql = 1.0, w = 1.0, pm = 1.0, p = c;
    g = 0.5 * (1.0 - c);
    f = 0.5;
#pragma unroll 1
    for (int l = 1; l <= kSbmL; ++l) {
        ql *= q;
        w *= ql;
        const double pn = kLegendre.a[l] * c * p - kLegendre.b[l] * pm;
        g = fma(0.5 * w, pm - pn, g);
        f = fma((l + 0.5) * w, p, f);
        pm = p;
        p = pn;
    }
}

// t >= kSbmSwitch: cos drawn exactly, P(cos <= c) = u, by Newton steps on
// the series kept inside a shrinking bisection bracket (at most 40 steps;
// a step that leaves the bracket or is NaN bisects instead); returns
// (cos, sin).  Rare: with the residual-range step on, t stays below ~2e-2
// on every full step.  Out of line, so that its double-precision registers
// never add to the step's: registers live across the call are saved only
// when it runs.
__device__ __noinline__ float2 sbm_large(float t, float u) {
    const double td = t, target = 1.0 - (double)u, q = exp(-td);
    double lo = -1.0, hi = 1.0;
    double c = fmin(fmax(fmax(1.0 + td * log((double)u), 2.0 * (double)u - 1.0), -1.0), 1.0);
#pragma unroll 1
    for (int it = 0; it < 40; ++it) {
        double g, f;
        sbm_tail(q, c, g, f);
        if (g > target) lo = c; else hi = c;
        double cn = c + (g - target) / f;
        if (!(cn > lo && cn < hi)) cn = 0.5 * (lo + hi);
        const bool done = fabs(cn - c) <= 1e-14;
        c = cn;
        if (done) break;
    }
    return make_float2((float)c, (float)sqrt(fmax((1.0 - c) * (1.0 + c), 0.0)));
}

// Turn unit d by (ct, st) about itself, azimuth (cp, sp) from b1 of the
// Duff et al. (JCGT 2017) orthonormal basis of d.
__device__ __forceinline__ void turn(float& dx, float& dy, float& dz, float ct, float st,
                                     float cp, float sp) {
    const float sg = copysignf(1.0f, dz);
    const float a = -frcp(sg + dz);   // |sg + dz| >= 1
    const float b = dx * dy * a;
    const float b1x = 1.0f + sg * dx * dx * a, b1y = sg * b, b1z = -sg * dx;
    const float b2x = b, b2y = sg + dy * dy * a, b2z = -dy;
    const float ex = cp * b1x + sp * b2x, ey = cp * b1y + sp * b2y, ez = cp * b1z + sp * b2z;
    const float nx = ct * dx + st * ex, ny = ct * dy + st * ey, nz = ct * dz + st * ez;
    dx = nx;
    dy = ny;
    dz = nz;
}

__device__ __forceinline__ bool inside(const KParams& P, float x, float y, float z) {
    return x >= P.lo[0] && x <= P.hi[0] && y >= P.lo[1] && y <= P.hi[1] && z >= P.lo[2] &&
           z <= P.hi[2];
}

// Voxel of an inside point; the upper face belongs to the last voxel.
__device__ __forceinline__ void voxel3(const KParams& P, float x, float y, float z, int& ix,
                                       int& iy, int& iz) {
    ix = min((int)((x - P.lo[0]) * P.inv_d[0]), P.nx - 1);
    iy = min((int)((y - P.lo[1]) * P.inv_d[1]), P.ny - 1);
    iz = min((int)((z - P.lo[2]) * P.inv_d[2]), P.nz - 1);
}

// Fixed-point energy, round to nearest even; e >= 0 always (deposits,
// energies), so the conversion is the unsigned one, without a sign fix-up.
__device__ __forceinline__ long long fixp(float e, float wsc) {
    return (long long)(unsigned long long)rintf(e * wsc);
}

// Per-lane deposit accumulator: consecutive deposits into the same voxel are
// summed in registers and written once when the voxel changes.  The voxel's
// coordinates are kept beside its linear index so that the tile test needs
// no division.
struct Acc {
    int v;
    int ix, iy, iz;
    long long q;
};

// Add the accumulated q: into the workgroup's LDS tile if the voxel lies in
// it, else into this XCD's replica of the global tally (hot lines then stay
// in one L2).
__device__ __forceinline__ void acc_flush(const KParams& P, unsigned long long* tile,
                                          unsigned long long* rep, Acc& a) {
    if (a.v >= 0 && a.q != 0) {
        const unsigned tx = (unsigned)(a.ix - P.tile_x0), ty = (unsigned)(a.iy - P.tile_y0),
                       tz = (unsigned)(a.iz - P.tile_z0);
        if (tx < (unsigned)P.tile_nx && ty < (unsigned)P.tile_ny && tz < (unsigned)P.tile_nz)
            atomicAdd(&tile[(tz * P.tile_ny + ty) * P.tile_nx + tx], (unsigned long long)a.q);
        else
            atomicAdd(&rep[a.v], (unsigned long long)a.q);
    }
    a.v = -1;
    a.q = 0;
}

// Score energy e at point (x,y,z): into the accumulator, or escaped.
// check = false skips the inside test where the caller knows the point is
// inside (a midpoint between two inside points of the box, with the
// monotonic rounding of fmaf).
__device__ __forceinline__ void score(const KParams& P, unsigned long long* tile,
                                      unsigned long long* rep, Acc& a, float x, float y, float z,
                                      float e, float wsc, long long& esc, bool check = true) {
    const long long q = fixp(e, wsc);
    if (check && !inside(P, x, y, z)) {
        esc += q;
        return;
    }
    int ix, iy, iz;
    voxel3(P, x, y, z, ix, iy, iz);
    const int v = (int)(((unsigned)iz * (unsigned)P.ny + (unsigned)iy) * (unsigned)P.nx +
                        (unsigned)ix);
    if (v == a.v) {
        a.q += q;
    } else {
        acc_flush(P, tile, rep, a);
        a.v = v;
        a.ix = ix;
        a.iy = iy;
        a.iz = iz;
        a.q = q;
    }
}

// Hydrogen (Mott) antiderivative in units of (eta/k)^2, Appendix A.2 with
// sin(eta ln((1+mu)/(1-mu))), and its derivative (the Mott cross section of
// section 2.1.4 in the same units).
__device__ __forceinline__ void mott_G_dG(float eta, float inv_2eta, float mu, float& G,
                                          float& dG) {
    const float omm = (1.0f - mu) * (1.0f + mu);
    const float iomm = frcp(omm);
    const float L = logf((1.0f + mu) * frcp(1.0f - mu));
    const float r = eta * L * 0.15915494309189535f;   // revolutions, |r| < 1 for E >= e_min
    const float sn = sin_rev(r), cs = cos_rev(r);
    G = 2.0f * mu * iomm - sn * inv_2eta;
    dG = 2.0f * iomm * ((1.0f + mu * mu) * iomm - 0.5f * cs);
}

// Invert the hydrogen elastic CDF, (G(mu) - G(lo)) / (G(hi) - G(lo)) = U, by
// Newton's method kept inside a shrinking bracket.  First guess: the
// interference term dropped, 2 mu / (1 - mu^2) = target.
__device__ __forceinline__ float mott_invert(const KParams& P, float eta, float U) {
    const float inv_2eta = 0.5f * frcp(eta);
    float a = P.mott_lo, b = P.mott_hi, G0, G1, d;
    mott_G_dG(eta, inv_2eta, a, G0, d);
    mott_G_dG(eta, inv_2eta, b, G1, d);
    const float tgt = fmaf(U, G1 - G0, G0);
    float mu = tgt * frcp(1.0f + sqrtf(1.0f + tgt * tgt));
    mu = fminf(fmaxf(mu, a), b);
    for (int it = 0; it < 24; ++it) {
        float G, dG;
        mott_G_dG(eta, inv_2eta, mu, G, dG);
        const float g = G - tgt;
        if (g < 0.0f) a = mu; else b = mu;
        float nx = mu - g * frcp(dG);
        if (!(nx > a && nx < b)) nx = 0.5f * (a + b);
        const float step = fabsf(nx - mu);
        mu = nx;
        // converged to a few ulps of mu (FP32 Newton can cycle between
        // neighbouring floats), or the bracket has closed
        if (step <= 2.5e-7f * fmaxf(fabsf(mu), 1e-3f) || !(b > a)) break;
    }
    return mu;
}

__device__ __forceinline__ float lerp_row(const float* row, int i, float f) {
    return fmaf(f, row[i + 1] - row[i], row[i]);
}

// Bilinear value of a [n_e][n_u] table at lattice (i, f) and x in [0, 1].
__device__ __forceinline__ float table_eu(const float* tab, int n_u, int i, float f, float x) {
    float tu = fminf(fmaxf(x * (float)(n_u - 1), 0.0f), (float)(n_u - 1));
    int j = min((int)tu, n_u - 2);
    const float g = tu - (float)j;
    const float* r0 = tab + (size_t)i * n_u;
    const float* r1 = r0 + n_u;
    const float a = fmaf(g, r0[j + 1] - r0[j], r0[j]);
    const float b = fmaf(g, r1[j + 1] - r1[j], r1[j]);
    return fmaf(f, b - a, a);
}

// Rate of channel (element e, elastic or inelastic) per cm at E.
__device__ __forceinline__ float channel_rate(const KParams& P, const ElemDev& d, bool inel,
                                              float rho, float inv_e2, float mott, int li,
                                              float lf) {
    if (!inel) return rho * d.el_coef * inv_e2 * (d.is_h ? mott : 1.0f);
    return rho * d.ne_coef * lerp_row(P.nuc_sigma + (size_t)d.tab * P.n_e, li, lf);
}

// One large-angle jump at energy E (the state energy E_n) in material md,
// Eq. (Npi): channel by its rate, CM cosine from its law (closed-form
// Rutherford inverse, Mott by Newton, Kalbach-Mann inverse), CM -> lab by
// Eq. (cm_to_lab).  Outputs the loss fraction u (0 for elastic), the lab
// polar (cos, sin) and the azimuth (cos, sin).
__device__ void jump(const KParams& P, const MatDev* md, float E, float rho, uint4 q,
                     float& u_loss, float& jc, float& js, float& jcp, float& jsp, unsigned flags) {
    const float tl = (flog(E) - P.ln_e_lo) * P.inv_dln;
    const int li = max(0, min((int)tl, P.n_e - 2));
    const float lf = tl - (float)li;
    const float inv_e2 = 1.0f / (E * E);
    const float eta = P.eta_pre * __builtin_amdgcn_rsqf(E);
    const bool el = (flags & kElastic) != 0, ne = (flags & kInelastic) != 0;
    const int nel = md->n_elem;
    float mott = 0.0f;
    if (el && md->c_mott != 0.0f) {
        const float k = 0.15915494309189535f;   // revolutions per radian
        mott = P.mott_D0 -
               (sin_rev(eta * P.mott_Lhi * k) - sin_rev(eta * P.mott_Llo * k)) / (2.0f * eta);
    }
    float tot = 0.0f;
    for (int e = 0; e < nel; ++e) {
        const ElemDev& d = md->el[e];
        if (el) tot += channel_rate(P, d, false, rho, inv_e2, mott, li, lf);
        if (ne && d.tab >= 0) tot += channel_rate(P, d, true, rho, inv_e2, mott, li, lf);
    }
    const float target = u_hi(q.x) * tot;
    float acc = 0.0f;
    int ce = -1, cin = 0;
    for (int e = 0; e < nel && ce < 0; ++e) {
        const ElemDev& d = md->el[e];
        if (el) {
            acc += channel_rate(P, d, false, rho, inv_e2, mott, li, lf);
            if (target < acc) { ce = e; cin = 0; break; }
        }
        if (ne && d.tab >= 0) {
            acc += channel_rate(P, d, true, rho, inv_e2, mott, li, lf);
            if (target < acc) { ce = e; cin = 1; break; }
        }
    }
    if (ce < 0) {   // rounding at the top end: the last channel with a rate
        ce = nel - 1;
        cin = (ne && md->el[ce].tab >= 0) ? 1 : 0;
    }
    const ElemDev& d = md->el[ce];
    float cmc, cms;
    u_loss = 0.0f;
    if (!cin) {
        const float U = u_hi(q.y);
        if (d.is_h) {
            cmc = mott_invert(P, eta, U);
            cms = sqrtf(fmaxf(0.0f, (1.0f - cmc) * (1.0f + cmc)));
        } else {
            const float om = 1.0f / fmaf(U, P.ruth_T - 0.5f, 0.5f);   // 1 - mu
            cmc = 1.0f - om;
            cms = sqrtf(om * (2.0f - om));
        }
    } else {
        const size_t off = (size_t)d.tab * P.n_e * P.n_u;
        float u = table_eu(P.nuc_u + off, P.n_u, li, lf, u_hi(q.y));
        u = fminf(fmaxf(u, 0.0f), 1.0f);
        u_loss = u;
        const float a = table_eu(P.nuc_a + off, P.n_u, li, lf, u);
        const float r = table_eu(P.nuc_r + off, P.n_u, li, lf, u);
        const float U = u_hi(q.w);
        float mu;
        if (a < 1e-6f) {
            mu = 2.0f * U - 1.0f;
        } else {
            const float sh = sinhf(a), ch = coshf(a);
            const float C = 2.0f * sh * U + r * ch - sh;
            mu = logf((C + sqrtf(C * C - r * r + 1.0f)) / (1.0f + r)) / a;
            mu = fminf(fmaxf(mu, -1.0f), 1.0f);
        }
        cmc = mu;
        cms = sqrtf(fmaxf(0.0f, (1.0f - mu) * (1.0f + mu)));
    }
    // CM -> lab (Appendix A.1): K = E, m1 = m_p, outgoing lab energy E - u E
    const float m1 = kMpF, m2 = d.m2;
    const float E1 = E + m1;
    const float p1 = sqrtf(E * (E + 2.0f * m1));
    const float ucm = p1 / (E1 + m2);
    const float gu = 1.0f / sqrtf((1.0f - ucm) * (1.0f + ucm));
    const float K2 = E * (1.0f - u_loss);
    const float E1p = K2 + m1;
    const float p1p = sqrtf(K2 * (K2 + 2.0f * m1));
    const float v1c = (p1p - ucm * E1p) / (E1p - ucm * p1p);
    const float X = gu * (cmc + ucm / v1c), Y = cms;
    const float rn = 1.0f / sqrtf(X * X + Y * Y);
    jc = X * rn;
    js = Y * rn;
    const float phi = u_hi(q.z);
    jcp = cos_rev(phi);
    jsp = sin_rev(phi);
}

// FP64 residual range R_g(E) (g/cm^2) by cubic Hermite on the lattice.
__device__ __forceinline__ double range_g64(const KParams& P, int mat, float E) {
    const double t = (log((double)E) - P.ln_e_lo_d) * P.inv_dln_d;
    int i = (int)floor(t);
    i = max(0, min(i, P.n_e - 2));
    const double s = t - (double)i;
    const double2 a = P.rg64[(size_t)mat * P.n_e + i];
    const double2 b = P.rg64[(size_t)mat * P.n_e + i + 1];
    const double s2 = s * s, s3 = s2 * s;
    return (2.0 * s3 - 3.0 * s2 + 1.0) * a.x + (s3 - 2.0 * s2 + s) * a.y +
           (-2.0 * s3 + 3.0 * s2) * b.x + (s3 - s2) * b.y;
}

// Per-history record {E0, steps, jumps, end, x, y, z, E, first jump step,
// last jump step, 0, 0}: end 1 = end of range, 2 = left the phantom,
// 3 = below e_min, 4 = step limit, 5 = source; E is the energy at the end
// event (before absorption).
__device__ __forceinline__ void record(const KParams& P, unsigned long long h, float e0,
                                      unsigned steps, unsigned jumps, int end, float x, float y,
                                      float z, float e, int j1, int j2) {
    if (!P.rec) return;
    float* r = P.rec + h * 12;
    r[0] = e0;
    r[1] = (float)steps;
    r[2] = (float)jumps;
    r[3] = (float)end;
    r[4] = x;
    r[5] = y;
    r[6] = z;
    r[7] = e;
    r[8] = (float)j1;
    r[9] = (float)j2;
    r[10] = 0.0f;
    r[11] = 0.0f;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

enum : int { kDead = 0, kStep = 1, kJump = 2 };

// kFixed != 0: the physics switches are that compile-time constant (the
// method, with either small-angle sampler), so their tests fold away; 0:
// read them from P.flags.
template <unsigned kFixed>
__global__ void __launch_bounds__(1024) k_transport(KParams P) {
    const unsigned flags = kFixed ? kFixed : P.flags;
    extern __shared__ __align__(16) unsigned char smem[];
    float4* tab = reinterpret_cast<float4*>(smem);
    const int ntab = P.n_mat * P.n_e;
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) tab[i] = P.hot[i];
    float4* matc = tab + ntab;   // per material {zoa, Bethe log offset, end-of-range screen, 0}
    for (int i = threadIdx.x; i < P.n_mat; i += blockDim.x)
        matc[i] = make_float4(P.mats[i].zoa, P.mats[i].log_pre, P.ec[i], 0.0f);
    unsigned long long* tile =
        reinterpret_cast<unsigned long long*>(smem + (size_t)(ntab + P.n_mat) * 16);
    const int tile_n = P.tile_nx * P.tile_ny * P.tile_nz;
    for (int i = threadIdx.x; i < tile_n; i += blockDim.x) tile[i] = 0ull;
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const uint32_t k0 = (uint32_t)P.seed, k1 = (uint32_t)(P.seed >> 32);
    // tally replica of this XCD (any choice is correct; this one keeps hot
    // lines in one L2)
    const unsigned xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15u;   // HW_REG_XCC_ID
    unsigned long long* rep = P.tally + (size_t)(xcc % (unsigned)P.n_rep) * P.rep_stride;
    Acc acc{-1, 0, 0, 0, 0};
    int state = kDead;
    bool more = true;   // wave-uniform: the work counter may still hold histories
    unsigned long long q_next = 0, q_end = 0;   // wave-local range of history indices

    unsigned long long h = 0;
    unsigned n = 0;
    float E = 0.0f, rx = 0.0f, ry = 0.0f, rz = 0.0f, ox = 0.0f, oy = 0.0f, oz = 1.0f, wsc = 0.0f;
    int vcache = -1, mat = 0;
    float rho = 1.0f, e0 = 0.0f;
    // pending jump: state energy, material, density and step index at the jump
    float ej = 0.0f, rhoj = 1.0f;
    int matj = 0;
    unsigned nj = 0;
    unsigned hj = 0;
    int j1 = -1, j2 = -1;
    long long l_esc = 0, l_nuc = 0, l_e0 = 0;
    unsigned l_steps = 0, l_jumps = 0, l_hist = 0;
    // small-angle turn of the last step still to draw (exact regime): time,
    // uniform, azimuth
    bool sbm_pend = false;
    float sbm_t = 0.0f, sbm_u = 0.0f, sbm_ph = 0.0f;

    for (;;) {
        if (state == kDead) acc_flush(P, tile, rep, acc);
        // ---------------- small-angle turns in the exact regime ----------------
        // Drawn here, where little is live, before the lane's pending jump
        // (if any) turns it and before its next step moves it.  A history that
        // ended in that step needs no direction.
        if ((flags & kSbm) && sbm_pend) {
            if (state != kDead) {
                const float2 cs = sbm_large(sbm_t, sbm_u);
                turn(ox, oy, oz, cs.x, cs.y, cos_rev(sbm_ph), sin_rev(sbm_ph));
                const float inv = __builtin_amdgcn_rsqf(ox * ox + oy * oy + oz * oz);
                ox *= inv;
                oy *= inv;
                oz *= inv;
            }
            sbm_pend = false;
        }
        // ---------------- refill idle lanes ----------------
        // History indices come from a wave-local range [q_next, q_end) that is
        // refilled a chunk at a time from the global counter (one atomic per
        // chunk); the range is wave-uniform.
        const unsigned long long dead = __ballot(state == kDead);
        const int ndead = __popcll(dead);
        if (more && (ndead >= P.refill || ndead == 64)) {
            const int leader = __ffsll((long long)dead) - 1;
            const unsigned long long lim = q_end < P.n_hist ? q_end : P.n_hist;
            const unsigned long long avail = q_next < lim ? lim - q_next : 0ull;
            unsigned long long base = 0;
            const bool claim = avail < (unsigned long long)ndead;
            if (claim) {
                if (lane == leader) base = atomicAdd(P.counter, (unsigned long long)P.claim_chunk);
                base = __shfl(base, leader);
            }
            if (state == kDead) {
                const unsigned long long rank = __popcll(dead & ((1ull << lane) - 1ull));
                const unsigned long long hh = rank < avail ? q_next + rank : base + (rank - avail);
                if (hh < P.n_hist) {
                    // Source: spot by cumulative count in claim order; the
                    // history's index h is its index in the caller's spot
                    // order.  Box-Muller pairs from block (h, 2^32-1, 0):
                    // (w0, w1) lateral, (w2, w3) energy.
                    n = 0;
                    int lo = 0, hi = P.n_spots - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (P.prefix[mid] <= hh) lo = mid; else hi = mid - 1;
                    }
                    const SpotDev sp = P.spots[lo];
                    h = sp.h0 + (hh - P.prefix[lo]);
                    const uint4 w = philox((uint32_t)h, (uint32_t)(h >> 32), 0xFFFFFFFFu, 0u, k0, k1);
                    const float rr = fsqrt(-2.0f * flog(u_hi(w.x)));
                    const float a1 = u_hi(w.y);
                    const float z1 = rr * cos_rev(a1), z2 = rr * sin_rev(a1);
                    const float z3 = fsqrt(-2.0f * flog(u_hi(w.z))) * cos_rev(u_hi(w.w));
                    E = sp.E * (1.0f + sp.sigmaE * z3);
                    rx = sp.x + sp.sxy * z1;
                    ry = sp.y + sp.sxy * z2;
                    rz = P.lo[2];
                    ox = 0.0f;
                    oy = 0.0f;
                    oz = 1.0f;
                    wsc = sp.wscale;
                    e0 = E;
                    hj = 0;
                    j1 = -1;
                    j2 = -1;
                    l_hist++;
                    l_e0 += fixp(E, wsc);
                    if (!inside(P, rx, ry, rz)) {
                        l_esc += fixp(E, wsc);
                        record(P, h, e0, 0, 0, 5, rx, ry, rz, E, -1, -1);
                    } else if (E < P.e_min) {
                        score(P, tile, rep, acc, rx, ry, rz, E, wsc, l_esc);
                        record(P, h, e0, 0, 0, 5, rx, ry, rz, E, -1, -1);
                    } else {
                        int ix, iy, iz;
                        voxel3(P, rx, ry, rz, ix, iy, iz);
                        vcache = (int)(((unsigned)iz * (unsigned)P.ny + (unsigned)iy) *
                                           (unsigned)P.nx + (unsigned)ix);
                        const uint2 pk = P.vox[vcache];
                        rho = __uint_as_float(pk.x);
                        mat = (int)pk.y;
                        state = kStep;
                    }
                }
            }
            if (claim) {
                q_next = base + ((unsigned long long)ndead - avail);
                q_end = base + (unsigned long long)P.claim_chunk;
                if (base >= P.n_hist) more = false;
            } else {
                q_next += (unsigned long long)ndead;
            }
        }
        if (!more && __ballot(state != kDead) == 0ull) break;

        // ---------------- finish pending jumps, a batch at a time ----------------
        const unsigned long long pend = __ballot(state == kJump);
        const unsigned long long stepping = __ballot(state == kStep);
        if (pend && ((int)__popcll(pend) >= P.jump_batch || stepping == 0ull)) {
            if (state == kJump) {
                const uint4 q = philox((uint32_t)h, (uint32_t)(h >> 32), nj, 1u, k0, k1);
                float u_loss, jc, js, jcp, jsp;
                jump(P, P.mats + matj, ej, rhoj, q, u_loss, jc, js, jcp, jsp, flags);
                // E holds E' (after continuous loss); the jump removes u E'
                const float En = E * (1.0f - u_loss);
                l_nuc += fixp(E, wsc) - fixp(En, wsc);
                E = En;
                turn(ox, oy, oz, jc, js, jcp, jsp);
                const float inv = __builtin_amdgcn_rsqf(ox * ox + oy * oy + oz * oz);
                ox *= inv;
                oy *= inv;
                oz *= inv;
                l_jumps++;
                hj++;
                if (j1 < 0) j1 = (int)nj;
                j2 = (int)nj;
                state = kStep;
                if (!inside(P, rx, ry, rz)) {
                    l_esc += fixp(E, wsc);
                    record(P, h, e0, n, hj, 2, rx, ry, rz, E, j1, j2);
                    state = kDead;
                } else if (E < P.e_min) {
                    score(P, tile, rep, acc, rx, ry, rz, E, wsc, l_esc);
                    record(P, h, e0, n, hj, 3, rx, ry, rz, E, j1, j2);
                    state = kDead;
                }
            }
        }
        if (state != kStep) continue;

        // ---------------- one step of Eq. (VSDE) ----------------
        if ((long long)n >= P.max_steps) {
            atomicAdd(&P.ledger[4], (unsigned long long)fixp(E, wsc));
            record(P, h, e0, n, hj, 4, rx, ry, rz, E, j1, j2);
            state = kDead;
            continue;
        }
        const float4 mc = matc[mat];

        // End of range: residual range within one step, decided in FP64; the
        // FP32 screen E <= ec(material) is exact-safe (ec bounds the energy
        // whose range fits a step at the densest voxel of that material).
        if ((flags & kEor) && E <= mc.z) {
            const double rres = range_g64(P, mat, E) / (double)rho;
            if (rres <= P.step_d) {
                const float hr = (float)(0.5 * rres);
                score(P, tile, rep, acc, fmaf(ox, hr, rx), fmaf(oy, hr, ry), fmaf(oz, hr, rz), E, wsc,
                      l_esc);
                l_steps++;
                const float fr = (float)rres;
                record(P, h, e0, n + 1, hj, 1, fmaf(ox, fr, rx), fmaf(oy, fr, ry),
                       fmaf(oz, fr, rz), E, j1, j2);
                state = kDead;
                continue;
            }
        }

        const float lnE = flog(E);
        const float tl = (lnE - P.ln_e_lo) * P.inv_dln;
        const int li = max(0, min((int)tl, P.n_e - 2));
        const float lf = tl - (float)li;
        const float4 ta = tab[mat * P.n_e + li], tb = tab[mat * P.n_e + li + 1];
        const uint4 w = philox((uint32_t)h, (uint32_t)(h >> 32), n, 0u, k0, k1);

        // Continuous loss, Eq. (bethbloch) with Bragg additivity; clamped
        // straggling, Eq. (energystraggling), B_n ~ N(0, Delta).
        const float p2 = E * (E + 2.0f * kMpF);
        const float g = E + kMpF;
        const float b2 = p2 * frcp(g * g);
        float s1 = 0.0f;
        if (flags & kLoss) {
            const float L = mc.y + flog(p2) - b2;
            s1 = rho * P.c_bethe * mc.x * L * frcp(b2);
        }
        const float a = s1 * P.step;
        float X = 0.0f;
        if (flags & kStraggle) {
            const float gm = g * (1.0f / kMpF);
            const float var = rho * P.c_strag * mc.x * gm * gm * (1.0f - 0.5f * b2);
            const float zE = fsqrt(-2.0f * flog(u_hi(w.x))) * cos_rev(u_hi(w.y));
            X = fminf(fmaxf(fsqrt(var) * P.sqrt_step * zE, -a), a);
        }
        const float Ep = fmaxf(E - a + X, 0.0f);

        // Jump test: none with probability exp(-Delta sigma).  Elastic rate
        // (Rutherford + Mott) = el_E2 / E^2 with el_E2 smooth in ln E;
        // inelastic rate linear on the lattice.
        bool jumped = false;
        if (flags & (kElastic | kInelastic)) {
            const float el_e2 = fmaf(lf, tb.w - ta.w, ta.w);
            const float ne_rate = fmaf(lf, tb.z - ta.z, ta.z);
            const float rate = ((flags & kElastic) ? el_e2 * frcp(E * E) : 0.0f) +
                               ((flags & kInelastic) ? ne_rate : 0.0f);
            const float lam = P.step * rho * rate;
            const float pj = lam < 0.05f
                ? lam * fmaf(-0.5f * lam, fmaf(-lam * (1.0f / 3.0f), fmaf(-0.25f, lam, 1.0f), 1.0f), 1.0f)
                : 1.0f - __expf(-lam);
            jumped = u_lo(w.x, w.y, w.z) < pj;
        }

        // Deposit E_n - E' at the step midpoint (pre-step direction), move.
        // Both R_n and, when in_next, R_{n+1} lie in the box, and so does the
        // midpoint: its inside test is needed only when R_{n+1} left.
        const float nx = fmaf(ox, P.step, rx), ny = fmaf(oy, P.step, ry), nz = fmaf(oz, P.step, rz);
        const bool in_next = inside(P, nx, ny, nz);
        score(P, tile, rep, acc, fmaf(ox, P.half_step, rx), fmaf(oy, P.half_step, ry),
              fmaf(oz, P.half_step, rz), E - Ep, wsc, l_esc, !in_next);
        rx = nx;
        ry = ny;
        rz = nz;
        uint2 pk_next = make_uint2(0u, 0u);
        int v_next = vcache;
        if (in_next) {   // prefetch the next voxel while the direction is updated
            int ix, iy, iz;
            voxel3(P, rx, ry, rz, ix, iy, iz);
            v_next = (int)(((unsigned)iz * (unsigned)P.ny + (unsigned)iy) * (unsigned)P.nx +
                           (unsigned)ix);
            if (v_next != vcache) pk_next = P.vox[v_next];
        }

        // Small-angle diffusion over time t = sigma^2 Delta / z, sigma the
        // Lynch-Dahl width: the spherical Brownian motion law (switch kSbm;
        // the lineage count's normal is the sine partner of Z_E's
        // Box-Muller pair) or the geodesic Gaussian step of per-axis
        // variance t.
        if (flags & kMcs) {
            const float A1 = fmaf(lf, tb.x - ta.x, ta.x);
            const float A2 = fmaf(lf, tb.y - ta.y, ta.y);
            const float nu = rho * A2;
            const float br = (1.0f + frcp(nu)) * flog(1.0f + nu) - 1.0f;
            const float sig2 = rho * A1 * br;
            float ct = 1.0f, st = 0.0f;
            bool now = true;
            if (flags & kSbm) {
                if (sig2 < kSbmSwitch) {
                    const float zM = fsqrt(-2.0f * flog(u_hi(w.x))) * sin_rev(u_hi(w.y));
                    sbm_small(sig2, zM, u_hi(w.z), ct, st);
                } else {   // exact regime: drawn at the top of the loop
                    now = false;
                    sbm_pend = true;
                    sbm_t = sig2;
                    sbm_u = u_hi(w.z);
                    sbm_ph = u_hi(w.w);
                }
            } else {
                polar_cs(-2.0f * sig2 * flog(u_hi(w.z)), ct, st);
            }
            if (now) {
                const float ph = u_hi(w.w);
                turn(ox, oy, oz, ct, st, cos_rev(ph), sin_rev(ph));
            }
        }
        l_steps++;
        if (jumped) {
            // the jump (and the renormalisation after it) is finished in a batch
            ej = E;
            matj = mat;
            rhoj = rho;
            nj = n;
            E = Ep;
            n++;
            state = kJump;
        } else {
            const float inv = __builtin_amdgcn_rsqf(ox * ox + oy * oy + oz * oz);
            ox *= inv;
            oy *= inv;
            oz *= inv;
            E = Ep;
            n++;
            if (!in_next) {
                l_esc += fixp(E, wsc);
                record(P, h, e0, n, hj, 2, rx, ry, rz, E, j1, j2);
                state = kDead;
            } else if (E < P.e_min) {
                score(P, tile, rep, acc, rx, ry, rz, E, wsc, l_esc);
                record(P, h, e0, n, hj, 3, rx, ry, rz, E, j1, j2);
                state = kDead;
            }
        }
        if (in_next && v_next != vcache) {
            rho = __uint_as_float(pk_next.x);
            mat = (int)pk_next.y;
            vcache = v_next;
        }
    }

    acc_flush(P, tile, rep, acc);
    // ledger: wave sums, one atomic per slot per wave
    const unsigned long long s_esc = wave_sum((unsigned long long)l_esc);
    const unsigned long long s_nuc = wave_sum((unsigned long long)l_nuc);
    const unsigned long long s_e0 = wave_sum((unsigned long long)l_e0);
    const unsigned long long s_st = wave_sum((unsigned long long)l_steps);
    const unsigned long long s_hi = wave_sum((unsigned long long)l_hist);
    const unsigned long long s_ju = wave_sum((unsigned long long)l_jumps);
    if (lane == 0) {
        atomicAdd(&P.ledger[1], s_esc);
        atomicAdd(&P.ledger[2], s_nuc);
        atomicAdd(&P.ledger[3], s_e0);
        atomicAdd(&P.ledger[5], s_st);
        atomicAdd(&P.ledger[6], s_hi);
        atomicAdd(&P.ledger[7], s_ju);
    }

    // flush the LDS tile
    __syncthreads();
    for (int i = threadIdx.x; i < tile_n; i += blockDim.x) {
        const unsigned long long q = tile[i];
        if (q) {
            const int tx = i % P.tile_nx, ty = (i / P.tile_nx) % P.tile_ny,
                      tz = i / (P.tile_nx * P.tile_ny);
            const size_t vv = ((size_t)(tz + P.tile_z0) * P.ny + (ty + P.tile_y0)) * P.nx +
                              (tx + P.tile_x0);
            atomicAdd(&rep[vv], q);
        }
    }
}

// Interleave density and material into one 8-byte word per voxel, count
// invalid voxels (material out of range, density not finite and positive)
// and record the largest density of each material (positive floats order
// like their bit patterns).
__global__ void k_pack(const uint8_t* mat, const float* rho, uint2* vox, size_t nvox, int n_mat,
                       unsigned int* bad, unsigned int* rho_max_bits) {
    unsigned rmax[kMaxMat];
#pragma unroll
    for (int m = 0; m < kMaxMat; ++m) rmax[m] = 0u;
    unsigned nbad = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvox;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint8_t m = mat[i];
        const float r = rho[i];
        const bool ok = (int)m < n_mat && r > 0.0f && r < 1e30f;
        nbad += ok ? 0u : 1u;
#pragma unroll
        for (int k = 0; k < kMaxMat; ++k)
            if (ok && (int)m == k) rmax[k] = max(rmax[k], __float_as_uint(r));
        vox[i] = make_uint2(__float_as_uint(ok ? r : 1.0f), ok ? (unsigned)m : 0u);
    }
    // one atomic per wave and slot
#pragma unroll
    for (int k = 0; k < kMaxMat; ++k) {
        unsigned v = rmax[k];
        for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, o));
        rmax[k] = v;
    }
    for (int o = 32; o > 0; o >>= 1) nbad += (unsigned)__shfl_xor((int)nbad, o);
    if ((threadIdx.x & 63) == 0) {
        if (nbad) atomicAdd(bad, nbad);
        for (int k = 0; k < n_mat && k < kMaxMat; ++k)
            if (rmax[k]) atomicMax(&rho_max_bits[k], rmax[k]);
    }
}

__global__ void k_reset(unsigned long long* tally, size_t nvox, unsigned long long* ledger,
                        unsigned long long* counter) {
    const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    for (size_t i = tid; i < nvox; i += (size_t)gridDim.x * blockDim.x) tally[i] = 0ull;
    if (tid < (size_t)kLedgerN) ledger[tid] = 0ull;
    if (tid == 0) *counter = 0ull;
}

// Dose to medium in FP64: E / (rho V), section 2.2.2; also sums the tally
// into the ledger's deposited slot (integer, order independent).
__global__ void __launch_bounds__(256) k_convert(unsigned long long* tally, int n_rep,
                                                 const uint2* vox, size_t nvox, double inv_scale,
                                                 double vcm3, double* dose,
                                                 unsigned long long* ledger) {
    unsigned long long s = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvox;
         i += (size_t)gridDim.x * blockDim.x) {
        unsigned long long q = tally[i];
        for (int r = 1; r < n_rep; ++r) q += tally[(size_t)r * nvox + i];
        if (n_rep > 1) tally[i] = q;   // replica 0 holds the total afterwards
        s += q;
        if (dose) {
            const double r = (double)__uint_as_float(vox[i].x);
            dose[i] = (double)(long long)q * inv_scale * kMevToJ / (r * vcm3 * 1e-3);
        }
    }
    s = wave_sum(s);
    __shared__ unsigned long long part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += part[k];
        atomicAdd(&ledger[0], t);
    }
}

int grid_for(size_t n, int block) {
    size_t g = (n + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

// The small-angle step's polar angle alone, for given times, uniforms and
// lineage normals (the same device functions as the transport), so that the
// sampler can be compared with another implementation value by value.
__global__ void k_sbm_polar(const float* __restrict__ t, const float* __restrict__ u,
                            const float* __restrict__ z, int n, float* __restrict__ c,
                            float* __restrict__ s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float ct, st;
    if (t[i] < kSbmSwitch) {
        sbm_small(t[i], z[i], u[i], ct, st);
    } else {
        const float2 cs = sbm_large(t[i], u[i]);
        ct = cs.x;
        st = cs.y;
    }
    c[i] = ct;
    s[i] = st;
}

}  // namespace

hipError_t launch_pack_phantom(const uint8_t* mat, const float* rho, uint2* vox, size_t nvox,
                               int n_mat, unsigned int* bad, unsigned int* rho_max_bits,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_pack, dim3(std::min(grid_for(nvox, 256), 4096)), dim3(256), 0, s, mat,
                       rho, vox, nvox,
                       n_mat, bad, rho_max_bits);
    return hipGetLastError();
}

hipError_t launch_sbm_polar(const float* t, const float* u, const float* z, int n, float* c,
                            float* s_out, hipStream_t s) {
    hipLaunchKernelGGL(k_sbm_polar, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t, u, z,
                       n, c, s_out);
    return hipGetLastError();
}

hipError_t launch_reset(unsigned long long* tally, size_t nvox, unsigned long long* ledger,
                        unsigned long long* counter, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(grid_for(nvox, 256)), dim3(256), 0, s, tally, nvox, ledger,
                       counter);
    return hipGetLastError();
}

hipError_t transport_kernel_attributes(size_t lds_bytes) {
    const void* fns[] = {reinterpret_cast<const void*>(&k_transport<kMethod>),
                         reinterpret_cast<const void*>(&k_transport<kMethodGeodesic>),
                         reinterpret_cast<const void*>(&k_transport<0u>)};
    for (const void* f : fns) {
        const hipError_t e =
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_transport(const KParams& p, int grid, int block, size_t lds_bytes,
                            hipStream_t s) {
    if (p.flags == kMethod)
        hipLaunchKernelGGL(k_transport<kMethod>, dim3(grid), dim3(block), lds_bytes, s, p);
    else if (p.flags == kMethodGeodesic)
        hipLaunchKernelGGL(k_transport<kMethodGeodesic>, dim3(grid), dim3(block), lds_bytes, s,
                           p);
    else
        hipLaunchKernelGGL(k_transport<0u>, dim3(grid), dim3(block), lds_bytes, s, p);
    return hipGetLastError();
}

hipError_t launch_convert(unsigned long long* tally, int n_rep, const uint2* vox, size_t nvox,
                          double inv_scale, double voxel_cm3, double* dose,
                          unsigned long long* ledger, hipStream_t s) {
    // a bounded grid keeps the per-block ledger atomics few
    const int grid = std::min(grid_for(nvox, 256), 2048);
    hipLaunchKernelGGL(k_convert, dim3(grid), dim3(256), 0, s, tally, n_rep, vox, nvox,
                       inv_scale, voxel_cm3, dose, ledger);
    return hipGetLastError();
}

}  // namespace sde

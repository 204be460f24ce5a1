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
//
// The stepping is written once over its real type R.  R = float is the
// production instance (hardware transcendentals, FP32 lattice tables in LDS,
// FP64 only for the end-of-range decision).  R = double evaluates every
// coefficient in double precision (the Lynch-Dahl width and the elastic rate
// from their formulas instead of the FP32 lattice), for runs that must agree
// with a double-precision reference history by history.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "sde_elastic.hpp"
#include "sde_index.hpp"
#include "sde_internal.hpp"

namespace sde {
namespace {

constexpr unsigned kLoss = 1u, kStraggle = 2u, kMcs = 4u, kElastic = 8u, kInelastic = 16u,
                   kEor = 32u, kSbm = 64u, kEcut = 256u;
// the method (every switch) and the method with the geodesic Gaussian step:
// each its own compiled instance, the rest share k_transport<float, 0> (switches
// read at run time)
constexpr unsigned kMethod = 127u, kMethodGeodesic = 63u;

constexpr float kMpF = (float)kMp;
constexpr float kLn2 = 0.69314718055994530942f;
constexpr double kTwoPi = 6.283185307179586476925286766559;

// Arithmetic of one precision.  float: the gfx950 hardware log2, sqrt,
// reciprocal, reciprocal square root and sin/cos in revolutions; double: the
// correctly rounded (or nearly) library functions.
template <class R>
struct RM;

template <>
struct RM<float> {
    static constexpr bool f64 = false;
    static __device__ __forceinline__ float lg(float x) { return __builtin_amdgcn_logf(x) * kLn2; }
    static __device__ __forceinline__ float sq(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
    // sin and cos of 2 pi u: the hardware takes revolutions
    static __device__ __forceinline__ float sinr(float u) { return __builtin_amdgcn_sinf(u); }
    static __device__ __forceinline__ float cosr(float u) { return __builtin_amdgcn_cosf(u); }
    static __device__ __forceinline__ float fma(float a, float b, float c) { return fmaf(a, b, c); }
    // IEEE library forms where the hardware approximations were not enough
    static __device__ __forceinline__ float lgx(float x) { return logf(x); }
    static __device__ __forceinline__ float sqx(float x) { return sqrtf(x); }
    static __device__ __forceinline__ float sinh(float x) { return sinhf(x); }
    static __device__ __forceinline__ float cosh(float x) { return coshf(x); }
};

template <>
struct RM<double> {
    static constexpr bool f64 = true;
    static __device__ __forceinline__ double lg(double x) { return ::log(x); }
    static __device__ __forceinline__ double sq(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double rsq(double x) { return 1.0 / ::sqrt(x); }
    static __device__ __forceinline__ double sinr(double u) { return ::sin(kTwoPi * u); }
    static __device__ __forceinline__ double cosr(double u) { return ::cos(kTwoPi * u); }
    static __device__ __forceinline__ double fma(double a, double b, double c) { return ::fma(a, b, c); }
    static __device__ __forceinline__ double lgx(double x) { return ::log(x); }
    static __device__ __forceinline__ double sqx(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double sinh(double x) { return ::sinh(x); }
    static __device__ __forceinline__ double cosh(double x) { return ::cosh(x); }
};

template <class R>
__device__ __forceinline__ const KScal<R>& scal(const KParams& P);
template <>
__device__ __forceinline__ const KScal<float>& scal<float>(const KParams& P) { return P.sf; }
template <>
__device__ __forceinline__ const KScal<double>& scal<double>(const KParams& P) { return P.sd; }

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

// (2k+1) 2^-24 from the top 23 bits: exact in FP32 and FP64, never 0 or 1.
template <class R>
__device__ __forceinline__ R u_hi(uint32_t w) { return ((R)(w >> 9) + R(0.5)) * R(0x1p-23); }
// Same from the 23 low bits that u_hi leaves unused in three words.
template <class R>
__device__ __forceinline__ R u_lo(uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t k = (a & 0x1FFu) | ((b & 0x1FFu) << 9) | ((c & 0x1Fu) << 18);
    return ((R)k + R(0.5)) * R(0x1p-23);
}

// cos and sin of a polar angle given its square.  float: Taylor in theta^2
// for small angles (where the hardware sine would lose relative accuracy),
// the hardware sine and cosine (absolute error ~1e-7) otherwise.
template <class R>
__device__ __forceinline__ void polar_cs(R th2, R& c, R& s) {
    if constexpr (RM<R>::f64) {
        const double th = ::sqrt(th2);
        c = ::cos(th);
        s = ::sin(th);
    } else {
        if (th2 < 0.25f) {
            const float x = th2;
            c = fmaf(x, fmaf(x, fmaf(x, fmaf(x, fmaf(x, -2.7557319e-7f, 2.4801587e-5f),
                                             -1.3888889e-3f), 4.1666667e-2f), -0.5f), 1.0f);
            const float sc = fmaf(x, fmaf(x, fmaf(x, fmaf(x, fmaf(x, -2.5052108e-8f, 2.7557319e-6f),
                                                  -1.9841270e-4f), 8.3333333e-3f),
                                          -1.6666667e-1f), 1.0f);
            s = RM<float>::sq(x) * sc;
        } else {
            const float r = sqrtf(th2) * 0.15915494309189535f;   // revolutions
            s = RM<float>::sinr(r);
            c = RM<float>::cosr(r);
        }
    }
}

// Spherical Brownian motion on S^2 (generator half the Laplace-Beltrami
// operator) at time t = sigma^2 Delta / z, the law of the small-angle
// diffusion over one step (section 2.1.4), by the sampler the paper cites
// (Mijatovic, Mramor and Uribe Bravo 2020, Algorithm 1): M = the number of
// lineages left at time t of Kingman's coalescent with mutation parameter
// d - 1 = 2 started from infinitely many, X ~ Beta(1, 1 + M),
// cos = 1 - 2 X.  u -> 1 gives the angle -> 0 in both regimes.
template <class R>
struct SbmSwitch;
template <>
struct SbmSwitch<float> { static constexpr float t = 0.02f; };
template <>
struct SbmSwitch<double> { static constexpr double t = 0.02; };
constexpr int kSbmL = 64;   // Legendre terms: e^{-l(l+1)t/2} < 1e-18 beyond, t >= 0.02

// t below the switch: M from Griffiths' normal law with mean 1/expm1(t/2)
// and its variance, rounded to the nearest integer and floored at 0; then
// X by inversion, X = -expm1(ln u / (1 + M)).
// float: mean 2/t - 1/2 + t/24 (series of 1/expm1(t/2), error t^3/5760),
// standard deviation sqrt(2/(3t)) (1 - 7t^2/480), and -expm1 as a degree-7
// polynomial: here 1 + M >= 67 (|z| <= 5.77) and -ln u <= 16.7, so
// |ln u / (1 + M)| <= 0.25 and the truncation is below 2e-9 relative.
// double: the mean and variance from their closed forms (the variance's
// bracket by its Taylor series below t = 1e-2, where it cancels).
template <class R>
__device__ __forceinline__ void sbm_small(R t, R z, R u, R& ct, R& st) {
    if constexpr (RM<R>::f64) {
        double var;
        if (t < 1e-2) {
            const double t2 = t * t;
            var = 2.0 / (3.0 * t) * (1.0 - 7.0 * t2 / 240.0 + 41.0 * t2 * t2 / 80640.0);
        } else {
            const double beta = 0.5 * t, eta = beta / ::expm1(beta);
            var = (2.0 * eta / t) * (eta + beta) * (eta + beta) *
                  (1.0 + eta / (eta + beta) - 2.0 * eta) / (beta * beta);
        }
        const double M = ::fmax(::floor(1.0 / ::expm1(0.5 * t) + ::sqrt(var) * z + 0.5), 0.0);
        const double X = -::expm1(::log(u) / (1.0 + M));
        ct = 1.0 - 2.0 * X;
        st = 2.0 * ::sqrt(X * (1.0 - X));
    } else {
        t = fmaxf(t, 1e-30f);
        const float r = __builtin_amdgcn_rsqf(t);
        const float mu = fmaf(2.0f * r, r, fmaf(t, 1.0f / 24.0f, -0.5f));
        const float sd = 0.81649658f * r * fmaf(-7.0f / 480.0f * t, t, 1.0f);
        const float M = fmaxf(rintf(fmaf(sd, z, mu)), 0.0f);
        const float y = RM<float>::lg(u) * RM<float>::rcp(M + 1.0f);
        const float p = fmaf(y, fmaf(y, fmaf(y, fmaf(y, fmaf(y, fmaf(y, 1.0f / 5040.0f, 1.0f / 720.0f),
                                                             1.0f / 120.0f), 1.0f / 24.0f),
                                             1.0f / 6.0f), 0.5f), 1.0f);
        const float X = -y * p;
        ct = fmaf(-2.0f, X, 1.0f);
        st = 2.0f * RM<float>::sq(X * (1.0f - X));
    }
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

template <class R>
struct CosSin {
    R c, s;
};

// t at or above the switch: cos drawn exactly, P(cos <= c) = u, by Newton
// steps on the series kept inside a shrinking bisection bracket (at most 40
// steps; a step that leaves the bracket or is NaN bisects instead); returns
// (cos, sin).  Rare: with the residual-range step on, t stays below ~2e-2
// on every full step.  Out of line, so that its double-precision registers
// never add to the step's: registers live across the call are saved only
// when it runs.
template <class R>
__device__ __noinline__ CosSin<R> sbm_large(double td, double ud) {
    const double target = 1.0 - ud, q = exp(-td);
    double lo = -1.0, hi = 1.0;
    double c = fmin(fmax(fmax(1.0 + td * log(ud), 2.0 * ud - 1.0), -1.0), 1.0);
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
    return CosSin<R>{(R)c, (R)sqrt(fmax((1.0 - c) * (1.0 + c), 0.0))};
}

// Turn unit d by (ct, st) about itself, azimuth (cp, sp) from b1 of the
// Duff et al. (JCGT 2017) orthonormal basis of d.
template <class R>
__device__ __forceinline__ void turn(R& dx, R& dy, R& dz, R ct, R st, R cp, R sp) {
    const R sg = copysign(R(1), dz);
    const R a = -RM<R>::rcp(sg + dz);   // |sg + dz| >= 1
    const R b = dx * dy * a;
    const R b1x = R(1) + sg * dx * dx * a, b1y = sg * b, b1z = -sg * dx;
    const R b2x = b, b2y = sg + dy * dy * a, b2z = -dy;
    const R ex = cp * b1x + sp * b2x, ey = cp * b1y + sp * b2y, ez = cp * b1z + sp * b2z;
    const R nx = ct * dx + st * ex, ny = ct * dy + st * ey, nz = ct * dz + st * ez;
    dx = nx;
    dy = ny;
    dz = nz;
}

template <class R>
__device__ __forceinline__ bool inside(const KScal<R>& S, R x, R y, R z) {
    return x >= S.lo[0] && x <= S.hi[0] && y >= S.lo[1] && y <= S.hi[1] && z >= S.lo[2] &&
           z <= S.hi[2];
}

// Voxel of an inside point; the upper face belongs to the last voxel.
// float multiplies by the reciprocal voxel size; double divides, as the
// definition floor((x - origin) / d) reads.
template <class R>
__device__ __forceinline__ void voxel3(const KParams& P, const KScal<R>& S, R x, R y, R z,
                                       int& ix, int& iy, int& iz) {
    if constexpr (RM<R>::f64) {
        ix = axis_voxel(x, S.lo[0], 0.0, S.d[0], P.nx);
        iy = axis_voxel(y, S.lo[1], 0.0, S.d[1], P.ny);
        iz = axis_voxel(z, S.lo[2], 0.0, S.d[2], P.nz);
    } else {
        ix = axis_voxel(x, S.lo[0], S.inv_d[0], 0.0f, P.nx);
        iy = axis_voxel(y, S.lo[1], S.inv_d[1], 0.0f, P.ny);
        iz = axis_voxel(z, S.lo[2], S.inv_d[2], 0.0f, P.nz);
    }
}

// Fixed-point energy, round to nearest even; e >= 0 always (deposits,
// energies), so the conversion is the unsigned one, without a sign fix-up.
__device__ __forceinline__ long long fixp(float e, float wsc) {
    return (long long)(unsigned long long)rintf(e * wsc);
}
__device__ __forceinline__ long long fixp(double e, double wsc) {
    return (long long)(unsigned long long)rint(e * wsc);
}

// Per-lane deposit accumulator: consecutive deposits into the same voxel are
// summed in registers, as weighted energy in the stepping precision, and
// written once, in fixed point, when the voxel changes.  The voxel's slot in
// the workgroup's LDS tile (-1 outside it) is found when the voxel is first
// scored, beside its linear index.
template <class R>
struct Acc {
    int v;
    int slot;
    R e;   // sum of e * wsc (fixed-point units)
};

// Add the accumulated energy, rounded to fixed point: into the workgroup's
// LDS tile if the voxel lies in it, else into this XCD's replica of the
// global tally (hot lines then stay in one L2).  The two atomics carry
// different scopes, so that they stay an LDS and a global instruction
// rather than one generic (flat) atomic on a selected address.
template <class R>
__device__ __forceinline__ void acc_flush(unsigned long long* tile, unsigned long long* rep,
                                          Acc<R>& a) {
    if (a.v >= 0 && a.e != R(0)) {
        const unsigned long long q = (unsigned long long)fixp(a.e, R(1));
        if (a.slot >= 0)
            __hip_atomic_fetch_add(&tile[a.slot], q, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            __hip_atomic_fetch_add(&rep[a.v], q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    a.v = -1;
    a.e = R(0);
}

// Score energy e at point (x,y,z): into the accumulator, or escaped.
// check = false skips the inside test where the caller knows the point is
// inside (a midpoint between two inside points of the box, with the
// monotonic rounding of fma).
template <class R>
__device__ __forceinline__ void score(const KParams& P, const KScal<R>& S,
                                      unsigned long long* tile, unsigned long long* rep, Acc<R>& a,
                                      R x, R y, R z, R e, R wsc, long long& esc,
                                      bool check = true) {
    if (check && !inside(S, x, y, z)) {
        esc += fixp(e, wsc);
        return;
    }
    const R eq = e * wsc;
    int ix, iy, iz;
    voxel3(P, S, x, y, z, ix, iy, iz);
    const int v = voxel_index(ix, iy, iz, P.nx, P.ny, P.nz);
    if (v == a.v) {
        a.e += eq;
    } else {
        acc_flush(tile, rep, a);
        a.v = v;
        a.slot = tile_slot(ix, iy, iz, P.tile_x0, P.tile_y0, P.tile_z0, P.tile_nx, P.tile_ny,
                           P.tile_nz);
        a.e = eq;
    }
}

// Hydrogen (Mott) antiderivative in units of (eta/k)^2, Appendix A.2 with
// sin(eta ln((1+mu)/(1-mu))), written in s = 1 - mu (which keeps the forward
// angles, s << 1, at full relative precision):
//   G(s) = 2 (1 - s) / (s (2 - s)) - sin(eta ln((2 - s) / s)) / (2 eta),
// and dG/ds, minus the Mott cross section of section 2.1.4 in the same units.
template <class R>
__device__ __forceinline__ void mott_G_dG(R eta, R inv_2eta, R s, R& G, R& dG) {
    using M = RM<R>;
    const R q = s * (R(2) - s);   // 1 - mu^2
    const R iq = M::rcp(q);
    const R L = M::lgx((R(2) - s) * M::rcp(s));
    const R r = eta * L * R(0.15915494309189535);   // revolutions, |r| < 1 for E >= e_min
    const R sn = M::sinr(r), cs = M::cosr(r);
    const R om = R(1) - s;
    G = R(2) * om * iq - sn * inv_2eta;
    dG = -R(2) * iq * ((R(1) + om * om) * iq - R(0.5) * cs);
}

// Invert the hydrogen elastic CDF in s: G(s) = G(s_lo) + U (G(s_hi) - G(s_lo))
// over [s_hi, s_lo] = [1 - cos(cut), 1 + cos(backscatter cut)], by Newton's
// method kept inside a shrinking bracket (G decreases in s).  First guess:
// the interference term dropped, 2 (1 - s) / (s (2 - s)) = target.
// Returns s = 1 - mu.
template <class R>
__device__ __forceinline__ R mott_invert(R s_hi, R s_lo, R eta, R U) {
    using M = RM<R>;
    // float: a few ulps of s (FP32 Newton can cycle between neighbouring
    // floats); double: 1e-15 of s
    constexpr R tol = M::f64 ? R(1e-15) : R(2.5e-7);
    constexpr int max_it = M::f64 ? 60 : 24;
    const R inv_2eta = R(0.5) * M::rcp(eta);
    R a = s_hi, b = s_lo, G0, G1, d;
    mott_G_dG(eta, inv_2eta, b, G0, d);
    mott_G_dG(eta, inv_2eta, a, G1, d);
    const R tgt = M::fma(U, G1 - G0, G0);
    R s = R(2) * M::rcp((tgt + R(1)) + M::sqx(tgt * tgt + R(1)));
    s = fmin(fmax(s, a), b);
    for (int it = 0; it < max_it; ++it) {
        R G, dG;
        mott_G_dG(eta, inv_2eta, s, G, dG);
        const R g = G - tgt;
        if (g > R(0)) a = s; else b = s;
        R nx = s - g * M::rcp(dG);
        if (!(nx > a && nx < b)) nx = R(0.5) * (a + b);
        const R step = fabs(nx - s);
        s = nx;
        // converged, or the bracket has closed
        if (step <= tol * s || !(b > a)) break;
    }
    return s;
}

template <class R>
__device__ __forceinline__ R lerp_row(const R* row, int i, R f) {
    return RM<R>::fma(f, row[i + 1] - row[i], row[i]);
}

// Bilinear value of a [n_e][n_u] table at lattice (i, f) and x in [0, 1].
template <class R>
__device__ __forceinline__ R table_eu(const R* tab, int n_u, int i, R f, R x) {
    using M = RM<R>;
    R tu = fmin(fmax(x * (R)(n_u - 1), R(0)), (R)(n_u - 1));
    int j = min((int)tu, n_u - 2);
    const R g = tu - (R)j;
    const R* r0 = tab + (size_t)i * n_u;
    const R* r1 = r0 + n_u;
    const R a = M::fma(g, r0[j + 1] - r0[j], r0[j]);
    const R b = M::fma(g, r1[j + 1] - r1[j], r1[j]);
    return M::fma(f, b - a, a);
}

// Per-precision views of a medium's jump constants and of the nuclear tables.
__device__ __forceinline__ int n_elem(const MatDev& m) { return m.n_elem; }
__device__ __forceinline__ int n_elem(const MatDev64& m) { return m.n_elem; }
__device__ __forceinline__ float el_coef(const MatDev& m, int e) { return m.el[e].el_coef; }
__device__ __forceinline__ double el_coef(const MatDev64& m, int e) { return m.el_coef[e]; }
__device__ __forceinline__ float el_base(const MatDev& m, int e) { return m.el[e].el_base; }
__device__ __forceinline__ double el_base(const MatDev64& m, int e) { return m.el_base[e]; }
__device__ __forceinline__ float ne_coef(const MatDev& m, int e) { return m.el[e].ne_coef; }
__device__ __forceinline__ double ne_coef(const MatDev64& m, int e) { return m.ne_coef[e]; }
__device__ __forceinline__ float m2_of(const MatDev& m, int e) { return m.el[e].m2; }
__device__ __forceinline__ double m2_of(const MatDev64& m, int e) { return m.m2[e]; }
__device__ __forceinline__ int is_h(const MatDev& m, int e) { return m.el[e].is_h; }
__device__ __forceinline__ int is_h(const MatDev64& m, int e) { return m.is_h[e]; }
__device__ __forceinline__ int tab_of(const MatDev& m, int e) { return m.el[e].tab; }
__device__ __forceinline__ int tab_of(const MatDev64& m, int e) { return m.tab[e]; }
__device__ __forceinline__ float c_mott(const MatDev& m) { return m.c_mott; }
__device__ __forceinline__ double c_mott(const MatDev64& m) { return m.c_mott; }

template <class R>
struct Nuc {
    const R *sigma, *u, *r, *a;
};
__device__ __forceinline__ Nuc<float> nuc_of(const KParams& P, float) {
    return Nuc<float>{P.nuc_sigma, P.nuc_u, P.nuc_r, P.nuc_a};
}
__device__ __forceinline__ Nuc<double> nuc_of(const KParams& P, double) {
    return Nuc<double>{P.nuc_sigma64, P.nuc_u64, P.nuc_r64, P.nuc_a64};
}

// Lynch-Dahl width of section 2.1.4 for the medium at density rho and
// energy E, scaled to the step: t = sigma^2 Delta / z (double instance).
__device__ __forceinline__ double ld_time64(const MatDev64& m, const KScal<double>& S, double rho,
                                            double E) {
    const double p2 = E * E + 2.0 * E * kMp;
    const double pb = p2 / (E + kMp);
    const double b2 = p2 / ((E + kMp) * (E + kMp));
    const double lp2 = ::log(p2);
    double wz = 0.0, num = 0.0;
    for (int i = 0; i < m.n_elem; ++i) {
        wz += m.wz[i];
        num += m.wz[i] * (m.ln_ca[i] + ::log1p(m.za2[i] / b2) - lp2);
    }
    const double chic2 = 0.157 * wz * rho * S.ld_z / (pb * pb);
    const double chia2 = ::exp(num / wz);
    const double nu = chic2 / (2.0 * chia2 * (1.0 - S.ld_F));
    const double s2 = chic2 / (1.0 + S.ld_F * S.ld_F) * ((1.0 + nu) / nu * ::log1p(nu) - 1.0);
    return s2 * (S.step / S.ld_z);
}

// The large-angle elastic cut in the forms the rates and samplers use:
// Rutherford T = 1 / (1 - cos), hydrogen's s_hi = 1 - cos, the rational and
// logarithmic terms of the Mott antiderivative at cos (D0 already less its
// value at the backscatter limit), and the cut itself.
template <class R>
struct Cut {
    R T, s_hi, D0, Lhi;
    R cos_r;   // cos of the cut for elements other than hydrogen (nuclear integrals)
};

template <class R>
__device__ __forceinline__ Cut<R> fixed_cut(const KScal<R>& S) {
    return Cut<R>{S.ruth_T, S.mott_shi, S.mott_D0, S.mott_Lhi, S.mott_hi};
}

// The cut 2.5 sigma for a Lynch-Dahl variance sig2z = sigma^2 at the width's
// path z, limited to pi (Rutherford) and pi - backscatter cut (hydrogen,
// where its interval closes); the half-angle forms keep small cuts exact.
template <class R>
__device__ __forceinline__ Cut<R> energy_cut(const KScal<R>& S, R sig2z) {
    using M = RM<R>;
    const R pi = R(3.14159265358979323846);
    const R th = fmin(R(2.5) * M::sq(sig2z), pi);
    const R th_h = fmin(th, pi - acos(-S.mott_lo));
    R hc, hs;
    polar_cs(R(0.25) * th * th, hc, hs);            // cos, sin of th / 2
    Cut<R> c;
    c.T = R(0.5) * M::rcp(hs * hs);                  // 1 / (1 - cos th)
    c.cos_r = hc * hc - hs * hs;
    polar_cs(R(0.25) * th_h * th_h, hc, hs);
    const R hs2 = hs * hs, hc2 = hc * hc;
    c.s_hi = R(2) * hs2;                             // 1 - cos th_h
    c.D0 = (hc2 - hs2) * M::rcp(R(2) * hs2 * hc2) - S.mott_Dlo;   // 2 cos / sin^2 - D(lo)
    c.Lhi = M::lgx(hc2 * M::rcp(hs2));               // ln((1 + cos) / (1 - cos))
    return c;
}

// The bracket of the hydrogen elastic rate: G(hi) - G(lo) of the Mott
// antiderivative in units of (eta/k)^2.
template <class R>
__device__ __forceinline__ R mott_bracket(const KScal<R>& S, const Cut<R>& c, R eta) {
    const R k = R(0.15915494309189535);   // revolutions per radian
    return c.D0 -
           (RM<R>::sinr(eta * c.Lhi * k) - RM<R>::sinr(eta * S.mott_Llo * k)) / (R(2) * eta);
}

// Lynch-Dahl variance sigma^2 at the width's path z for medium mat at
// density rho and energy E (lattice position li, lf): float from the FP32
// lattice rows, double from the formula.
template <class R>
__device__ __forceinline__ R ld_sig2z(const KParams& P, const KScal<R>& S, const float4* tab,
                                      int mat, R rho, R E, int li, R lf) {
    if constexpr (RM<R>::f64) {
        return ld_time64(P.mats64[mat], S, rho, E) * S.z_over_step;
    } else {
        const float4 ta = tab[mat * P.n_e + li], tb = tab[mat * P.n_e + li + 1];
        const float A1 = fmaf(lf, tb.x - ta.x, ta.x);
        const float A2 = fmaf(lf, tb.y - ta.y, ta.y);
        const float nu = rho * A2;
        const float br = (1.0f + RM<float>::rcp(nu)) * RM<float>::lg(1.0f + nu) - 1.0f;
        return rho * A1 * br * S.z_over_step;
    }
}

// ---- elastic nuclear terms (section 2.1.4) ----
__device__ __forceinline__ int ni_row(const MatDev& m, int e) { return m.el[e].ni; }
__device__ __forceinline__ int ni_row(const MatDev64& m, int e) { return m.ni[e]; }
__device__ __forceinline__ int h_nuc(const MatDev& m, int e) { return m.el[e].hn; }
__device__ __forceinline__ int h_nuc(const MatDev64& m, int e) { return m.hn[e]; }
__device__ __forceinline__ float nuc_coef(const MatDev& m, int e) { return m.el[e].nuc_coef; }
__device__ __forceinline__ double nuc_coef(const MatDev64& m, int e) { return m.nuc_coef[e]; }

template <class R>
struct NiTab {
    const R *p, *cum, *sig;
};
__device__ __forceinline__ NiTab<float> ni_of(const KParams& P, float) {
    return NiTab<float>{P.ni_p, P.ni_cum, P.ni_sig};
}
__device__ __forceinline__ NiTab<double> ni_of(const KParams& P, double) {
    return NiTab<double>{P.ni_p64, P.ni_cum64, P.ni_sig64};
}

// sigma_NI P_NI of table row t at lattice position (li, lf) and cosine x:
// its density and its integral from -1 to x, linear in the lattice
// coordinate between the two lattice energies.
template <class R>
__device__ __forceinline__ void ni_term(const KParams& P, int t, int li, R lf, R x, R& dens,
                                        R& integ) {
    const NiTab<R> T = ni_of(P, R(0));
    const int m = P.n_mu - 3;
    const size_t r0 = (size_t)t * P.n_e + li;
    R d0, i0, d1, i1;
    ni_spline(T.p + r0 * P.n_mu, T.cum + r0 * (P.n_mu - 2), m, x, d0, i0);
    ni_spline(T.p + (r0 + 1) * P.n_mu, T.cum + (r0 + 1) * (P.n_mu - 2), m, x, d1, i1);
    const R s0 = T.sig[r0], s1 = T.sig[r0 + 1];
    dens = (R(1) - lf) * s0 * d0 + lf * s1 * d1;
    integ = (R(1) - lf) * s0 * i0 + lf * s1 * i1;
}

// What the out-of-line hydrogen functions read, passed by value (a reference
// to the kernel's argument block cannot leave the kernel).
struct HTab {
    const double* coef;   // [3][n_l][n_e + 2]
    int n_l, n_e;
    double ln_e_lo, inv_dln, eta_pre;
};
__device__ __forceinline__ HTab h_tab(const KParams& P) {
    return HTab{P.h_coef, P.n_l, P.n_e, P.sd.ln_e_lo, P.sd.inv_dln, P.sd.eta_pre};
}

// Hydrogen's amplitudes at lattice coordinate tl (cubic B-splines, knots at
// the lattice points).
__device__ __forceinline__ HAmp h_amp(const HTab& P, double tl) {
    HAmp a;
    a.n_l = P.n_l;
    const int m = P.n_e - 1;
    double t = fmin(fmax(tl, 0.0), (double)m);
    int k = (int)floor(t);
    if (k > m - 1) k = m - 1;
    const double u = t - k, v = 1.0 - u;
    const double B0 = v * v * v / 6.0, B1 = (3.0 * u * u * u - 6.0 * u * u + 4.0) / 6.0,
                 B2 = (-3.0 * u * u * u + 3.0 * u * u + 3.0 * u + 1.0) / 6.0, B3 = u * u * u / 6.0;
    const size_t nc = (size_t)P.n_l * (P.n_e + 2);
    for (int l = 0; l < P.n_l; ++l) {
        const double* c = P.coef + (size_t)l * (P.n_e + 2) + k;
        a.are[l] = c[0] * B0 + c[1] * B1 + c[2] * B2 + c[3] * B3;
        a.aim[l] = c[nc] * B0 + c[nc + 1] * B1 + c[nc + 2] * B2 + c[nc + 3] * B3;
        a.b[l] = c[2 * nc] * B0 + c[2 * nc + 1] * B1 + c[2 * nc + 2] * B2 + c[2 * nc + 3] * B3;
    }
    return a;
}

// Integral (barn) of hydrogen's nuclear term over [lo, hi] at energy E,
// in double precision (its antiderivative cancels strongly); out of line.
__device__ __noinline__ double h_bracket64(HTab P, double E, double hi, double lo) {
    if (!(hi > lo)) return 0.0;
    const double tl = (log(E) - P.ln_e_lo) * P.inv_dln;
    const HAmp a = h_amp(P, tl);
    const double eta = P.eta_pre / sqrt(E);
    double d, g1, g0;
    h_nuclear(a, eta, hi, d, g1);
    h_nuclear(a, eta, lo, d, g0);
    return g1 - g0;
}

// The CM cosine's s = 1 - mu of a hydrogen elastic jump with the nuclear
// term: the distribution function of the summed cross section,
// ab G_mott(s) + nc G_N(1 - s) (ab = the Mott coefficient / E^2, nc = the
// nuclear coefficient), inverted over [s_hi, s_lo] by Newton's method in
// double precision kept inside a shrinking bracket; out of line.
__device__ __noinline__ double h_invert64(HTab P, double E, double ab, double nc, double s_hi,
                                          double s_lo, double U) {
    const double tl = (log(E) - P.ln_e_lo) * P.inv_dln;
    const HAmp A = h_amp(P, tl);
    const double eta = P.eta_pre / sqrt(E), inv_2eta = 0.5 / eta;
    auto G = [&](double s, double& dG) {
        double gm, dgm, dn, gn;
        mott_G_dG(eta, inv_2eta, s, gm, dgm);
        h_nuclear(A, eta, 1.0 - s, dn, gn);
        dG = ab * dgm - nc * dn;
        return ab * gm + nc * gn;
    };
    double d;
    const double G0 = G(s_lo, d), G1 = G(s_hi, d);
    const double tgt = G0 + U * (G1 - G0);
    double a = s_hi, b = s_lo, s = 0.5 * (s_hi + s_lo);
    for (int it = 0; it < 80; ++it) {
        double dG;
        const double g = G(s, dG) - tgt;
        if (g > 0.0) a = s; else b = s;
        double nx = s - g / dG;
        if (!(nx > a && nx < b)) nx = 0.5 * (a + b);
        const double step = fabs(nx - s);
        s = nx;
        if (step <= 1e-15 * s || !(b > a)) break;
    }
    return s;
}

// The same for an element other than hydrogen with sigma_NI P_NI:
// ab (1/s - 1/2) + nc NI(1 - s) over [s_c, 2], in the stepping precision.
template <class R>
__device__ R ni_invert(const KParams& P, int t, int li, R lf, R ab, R nc, R s_c, R U) {
    using M = RM<R>;
    constexpr R tol = M::f64 ? R(1e-15) : R(2.5e-7);
    constexpr int max_it = M::f64 ? 80 : 40;
    auto G = [&](R s, R& dG) {
        R dn, in;
        ni_term(P, t, li, lf, R(1) - s, dn, in);
        dG = -(ab * M::rcp(s * s) + nc * dn);
        return ab * (M::rcp(s) - R(0.5)) + nc * in;
    };
    R d;
    const R tgt = U * G(s_c, d);
    R a = s_c, b = R(2), s = fmin(s_c * R(2), R(1));
    for (int it = 0; it < max_it; ++it) {
        R dG;
        const R g = G(s, dG) - tgt;
        if (g > R(0)) a = s; else b = s;
        R nx = s - g / dG;
        if (!(nx > a && nx < b)) nx = R(0.5) * (a + b);
        const R step = fabs(nx - s);
        s = nx;
        if (step <= tol * s || !(b > a)) break;
    }
    return s;
}

// Nuclear elastic rate / rho of element e at E with the cut c: nc times the
// integral of its nuclear term over the law's range; hbr: hydrogen's
// bracket, computed once per medium by the caller.
template <class R, class Mat>
__device__ __forceinline__ R nuclear_rate(const KParams& P, const Mat& md, int e, int li, R lf,
                                          const Cut<R>& c, R hbr) {
    const int t = ni_row(md, e);
    if (t >= 0) {
        R d, in;
        ni_term(P, t, li, lf, c.cos_r, d, in);
        return nuc_coef(md, e) * in;
    }
    if (h_nuc(md, e)) return nuc_coef(md, e) * hbr;
    return R(0);
}

// Sum over the medium's elements of the nuclear elastic rates / rho at E
// with the cut c (0 without nuclear data).
template <class R, class Mat>
__device__ __forceinline__ R nuclear_sum(const KParams& P, const KScal<R>& S, const Mat& md, R E,
                                         int li, R lf, const Cut<R>& c) {
    R sum = R(0);
    if (P.n_ni == 0 && P.n_l == 0) return sum;
    for (int e = 0; e < n_elem(md); ++e) {
        R hbr = R(0);
        if (h_nuc(md, e))
            hbr = (R)h_bracket64(h_tab(P), (double)E, 1.0 - (double)c.s_hi, (double)S.mott_lo);
        sum += nuclear_rate(P, md, e, li, lf, c, hbr);
    }
    return sum;
}

// Rate of channel (element e, elastic or inelastic) per cm at E; ecut: the
// elastic coefficient at the cut c instead of the fixed one.
template <bool NUC, class R, class Mat>
__device__ __forceinline__ R channel_rate(const KParams& P, const Nuc<R>& nu, const Mat& m, int e,
                                          bool inel, R rho, R inv_e2, R mott, int li, R lf,
                                          bool ecut, const Cut<R>& c, R hbr) {
    if (!inel) {
        R nuc = R(0);
        if constexpr (NUC) nuc = nuclear_rate(P, m, e, li, lf, c, hbr);
        if (is_h(m, e)) return rho * (el_coef(m, e) * inv_e2 * mott + nuc);
        return rho * ((ecut ? el_base(m, e) * (c.T - R(0.5)) : el_coef(m, e)) * inv_e2 + nuc);
    }
    return rho * ne_coef(m, e) * lerp_row(nu.sigma + (size_t)tab_of(m, e) * P.n_e, li, lf);
}

// One large-angle jump at energy E (the state energy E_n) in medium md,
// Eq. (Npi): channel by its rate, CM cosine from its law (closed-form
// Rutherford inverse, Mott by Newton, Kalbach-Mann inverse), CM -> lab by
// Eq. (cm_to_lab).  Outputs the loss fraction u (0 for elastic), the lab
// polar (cos, sin) and the azimuth (cos, sin).  NUC: the instance carries the
// elastic nuclear terms (the general and FP64 instances; the method's own
// instances are launched only without such data).
template <bool NUC, class R, class Mat>
__device__ void jump(const KParams& P, const KScal<R>& S, const float4* tab, const Mat& md,
                     int mat, R E, R rho, uint4 q, R& u_loss, R& jc, R& js, R& jcp, R& jsp,
                     unsigned flags) {
    using M = RM<R>;
    const Nuc<R> nu = nuc_of(P, R(0));
    const R tl = (M::lg(E) - S.ln_e_lo) * S.inv_dln;
    const int li = lattice_interval(tl, P.n_e);
    const R lf = tl - (R)li;
    const R inv_e2 = R(1) / (E * E);
    const R eta = S.eta_pre * M::rsq(E);
    const bool el = (flags & kElastic) != 0, ne = (flags & kInelastic) != 0;
    const bool ecut = (flags & kEcut) != 0;
    const Cut<R> cut = (el && ecut) ? energy_cut(S, ld_sig2z(P, S, tab, mat, rho, E, li, lf))
                                    : fixed_cut(S);
    const int nel = n_elem(md);
    R mott = R(0), hbr = R(0);
    if (el && c_mott(md) != R(0)) mott = mott_bracket(S, cut, eta);
    if constexpr (NUC)
        if (el && P.n_l > 0)   // hydrogen's nuclear bracket, once
            for (int e = 0; e < nel; ++e)
                if (h_nuc(md, e))
                    hbr = (R)h_bracket64(h_tab(P), (double)E, 1.0 - (double)cut.s_hi,
                                     (double)S.mott_lo);
    R tot = R(0);
    for (int e = 0; e < nel; ++e) {
        if (el)
            tot += channel_rate<NUC>(P, nu, md, e, false, rho, inv_e2, mott, li, lf, ecut, cut, hbr);
        if (ne && tab_of(md, e) >= 0)
            tot += channel_rate<NUC>(P, nu, md, e, true, rho, inv_e2, mott, li, lf, ecut, cut, hbr);
    }
    const R target = u_hi<R>(q.x) * tot;
    R acc = R(0);
    int ce = -1, cin = 0;
    for (int e = 0; e < nel && ce < 0; ++e) {
        if (el) {
            acc += channel_rate<NUC>(P, nu, md, e, false, rho, inv_e2, mott, li, lf, ecut, cut, hbr);
            if (target < acc) { ce = e; cin = 0; break; }
        }
        if (ne && tab_of(md, e) >= 0) {
            acc += channel_rate<NUC>(P, nu, md, e, true, rho, inv_e2, mott, li, lf, ecut, cut, hbr);
            if (target < acc) { ce = e; cin = 1; break; }
        }
    }
    if (ce < 0) {   // rounding at the top end: the last channel with a rate
        ce = nel - 1;
        cin = (ne && tab_of(md, ce) >= 0) ? 1 : 0;
    }
    R cmc, cms;
    u_loss = R(0);
    if (!cin) {
        const R U = u_hi<R>(q.y);
        if (NUC && is_h(md, ce) && h_nuc(md, ce)) {
            // Mott + nuclear term: the summed law in double precision
            double sm = 0.0;
            if constexpr (NUC) sm = h_invert64(h_tab(P), (double)E, (double)(el_coef(md, ce) * inv_e2),
                                         (double)nuc_coef(md, ce), (double)cut.s_hi,
                                         (double)S.mott_slo, (double)U);
            cmc = (R)(1.0 - sm);
            cms = (R)sqrt(fmax(0.0, sm * (2.0 - sm)));
        } else if (is_h(md, ce)) {
            const R sm = mott_invert(cut.s_hi, S.mott_slo, eta, U);   // 1 - mu
            cmc = R(1) - sm;
            cms = M::sqx(fmax(R(0), sm * (R(2) - sm)));
        } else if (NUC && ni_row(md, ce) >= 0) {
            // Rutherford + sigma_NI P_NI: the summed law
            const R ab = el_base(md, ce) * inv_e2;
            R sm = R(1);
            if constexpr (NUC)
                sm = ni_invert(P, ni_row(md, ce), li, lf, ab, nuc_coef(md, ce), R(1) / cut.T, U);
            cmc = R(1) - sm;
            cms = M::sqx(fmax(R(0), sm * (R(2) - sm)));
        } else {
            const R om = R(1) / M::fma(U, cut.T - R(0.5), R(0.5));   // 1 - mu
            cmc = R(1) - om;
            cms = M::sqx(om * (R(2) - om));
        }
    } else {
        const size_t off = (size_t)tab_of(md, ce) * P.n_e * P.n_u;
        R u = table_eu(nu.u + off, P.n_u, li, lf, u_hi<R>(q.y));
        u = fmin(fmax(u, R(0)), R(1));
        u_loss = u;
        const R a = table_eu(nu.a + off, P.n_u, li, lf, u);
        const R r = table_eu(nu.r + off, P.n_u, li, lf, u);
        const R U = u_hi<R>(q.w);
        R mu;
        if (a < R(1e-6)) {
            mu = R(2) * U - R(1);
        } else {
            const R sh = M::sinh(a), ch = M::cosh(a);
            const R C = R(2) * sh * U + r * ch - sh;
            mu = M::lgx((C + M::sqx(C * C - r * r + R(1))) / (R(1) + r)) / a;
            mu = fmin(fmax(mu, R(-1)), R(1));
        }
        cmc = mu;
        cms = M::sqx(fmax(R(0), (R(1) - mu) * (R(1) + mu)));
    }
    // CM -> lab (Appendix A.1): K = E, m1 = m_p, outgoing lab energy E - u E
    const R m1 = (R)kMp, m2 = m2_of(md, ce);
    const R E1 = E + m1;
    const R p1 = M::sqx(E * (E + R(2) * m1));
    const R ucm = p1 / (E1 + m2);
    const R gu = R(1) / M::sqx((R(1) - ucm) * (R(1) + ucm));
    const R K2 = E * (R(1) - u_loss);
    const R E1p = K2 + m1;
    const R p1p = M::sqx(K2 * (K2 + R(2) * m1));
    const R v1c = (p1p - ucm * E1p) / (E1p - ucm * p1p);
    const R X = gu * (cmc + ucm / v1c), Y = cms;
    const R rn = R(1) / M::sqx(X * X + Y * Y);
    jc = X * rn;
    js = Y * rn;
    const R phi = u_hi<R>(q.z);
    jcp = M::cosr(phi);
    jsp = M::sinr(phi);
}

// FP64 residual range R_g(E) (g/cm^2) by cubic Hermite on the lattice.
__device__ __forceinline__ double range_g64(const KParams& P, int mat, double E) {
    const double t = (log(E) - P.sd.ln_e_lo) * P.sd.inv_dln;
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

enum : int { kDead = 0, kStep = 1, kJump = 2, kEnd = 3 };

__device__ __forceinline__ const SpotDev& spot_at(const KParams& P, int i, float) {
    return P.spots[i];
}
__device__ __forceinline__ const SpotDev64& spot_at(const KParams& P, int i, double) {
    return P.spots64[i];
}

// kFixed != 0: the physics switches are that compile-time constant (the
// method, with either small-angle sampler), so their tests fold away; 0:
// read them from P.flags.  kNuc: the elastic nuclear terms are compiled in
// (their double-precision hydrogen functions are out of line, and the calls
// cost registers, so only the instances launched with such data have them).
template <class R, unsigned kFixed, bool kNuc>
__global__ void __launch_bounds__(1024) k_transport(KParams P) {
    using M = RM<R>;
    const KScal<R>& S = scal<R>(P);
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
    Acc<R> acc{-1, -1, R(0)};
    int state = kDead;
    bool end_checked = false;   // the residual range exceeded the step: skip the screen once
    bool more = true;   // wave-uniform: the work counter may still hold histories
    unsigned long long q_next = 0, q_end = 0;   // wave-local range of history indices

    unsigned long long h = 0;
    unsigned n = 0;
    R E = R(0), rx = R(0), ry = R(0), rz = R(0), ox = R(0), oy = R(0), oz = R(1), wsc = R(0);
    int vcache = -1, mat = 0;
    R rho = R(1), e0 = R(0);
    // pending jump: state energy, material, density and step index at the jump
    R ej = R(0), rhoj = R(1);
    int matj = 0;
    unsigned nj = 0;
    unsigned hj = 0;
    int j1 = -1, j2 = -1;
    long long l_esc = 0, l_nuc = 0, l_e0 = 0, l_bad = 0;
    unsigned l_steps = 0, l_jumps = 0, l_hist = 0;
    // small-angle turn of the last step still to draw (exact regime): time,
    // uniform, azimuth
    bool sbm_pend = false;
    R sbm_t = R(0), sbm_u = R(0), sbm_ph = R(0);

    for (;;) {
        if (state == kDead) acc_flush(tile, rep, acc);
        // ---------------- small-angle turns in the exact regime ----------------
        // Drawn here, where little is live, before the lane's pending jump
        // (if any) turns it and before its next step moves it.  A history that
        // ended in that step needs no direction.
        if ((flags & kSbm) && sbm_pend) {
            if (state != kDead) {
                const CosSin<R> cs = sbm_large<R>((double)sbm_t, (double)sbm_u);
                turn(ox, oy, oz, cs.c, cs.s, M::cosr(sbm_ph), M::sinr(sbm_ph));
                const R inv = M::rsq(ox * ox + oy * oy + oz * oz);
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
                    const SpotT<R> sp = spot_at(P, lo, R(0));
                    h = sp.h0 + (hh - P.prefix[lo]);
                    const uint4 w = philox((uint32_t)h, (uint32_t)(h >> 32), 0xFFFFFFFFu, 0u, k0, k1);
                    const R rr = M::sq(R(-2) * M::lg(u_hi<R>(w.x)));
                    const R a1 = u_hi<R>(w.y);
                    const R z1 = rr * M::cosr(a1), z2 = rr * M::sinr(a1);
                    const R z3 = M::sq(R(-2) * M::lg(u_hi<R>(w.z))) * M::cosr(u_hi<R>(w.w));
                    E = sp.E * (R(1) + sp.sigmaE * z3);
                    rx = sp.x + sp.sxy * z1;
                    ry = sp.y + sp.sxy * z2;
                    rz = S.lo[2];
                    ox = R(0);
                    oy = R(0);
                    oz = R(1);
                    if (h == P.nan_h) ox = (R)__builtin_nan("");   // host-set test hook
                    wsc = sp.wscale;
                    e0 = E;
                    hj = 0;
                    j1 = -1;
                    j2 = -1;
                    l_hist++;
                    l_e0 += fixp(E, wsc);
                    if (!inside(S, rx, ry, rz)) {
                        l_esc += fixp(E, wsc);
                        record(P, h, (float)e0, 0, 0, 5, (float)rx, (float)ry, (float)rz, (float)E,
                               -1, -1);
                    } else if (E < S.e_min) {
                        score(P, S, tile, rep, acc, rx, ry, rz, E, wsc, l_esc);
                        record(P, h, (float)e0, 0, 0, 5, (float)rx, (float)ry, (float)rz, (float)E,
                               -1, -1);
                    } else {
                        int ix, iy, iz;
                        voxel3(P, S, rx, ry, rz, ix, iy, iz);
                        vcache = voxel_index(ix, iy, iz, P.nx, P.ny, P.nz);
                        const uint2 pk = P.vox[vcache];
                        rho = (R)__uint_as_float(pk.x);
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
                R u_loss, jc, js, jcp, jsp;
                if constexpr (M::f64)
                    jump<kNuc>(P, S, tab, P.mats64[matj], matj, ej, rhoj, q, u_loss, jc,
                                       js, jcp, jsp, flags);
                else
                    jump<kNuc>(P, S, tab, P.mats[matj], matj, ej, rhoj, q, u_loss, jc,
                                       js, jcp, jsp, flags);
                // E holds E' (after continuous loss); the jump removes u E'
                const R En = E * (R(1) - u_loss);
                turn(ox, oy, oz, jc, js, jcp, jsp);
                const R inv = M::rsq(ox * ox + oy * oy + oz * oz);
                ox *= inv;
                oy *= inv;
                oz *= inv;
                l_jumps++;
                hj++;
                if (j1 < 0) j1 = (int)nj;
                j2 = (int)nj;
                state = kStep;
                if (!__builtin_isfinite(En * ox)) {   // the lane guard, as after a step
                    l_bad += fixp(E, wsc);
                    record(P, h, (float)e0, n, hj, 6, (float)rx, (float)ry, (float)rz, (float)E,
                           j1, j2);
                    state = kDead;
                } else {
                    l_nuc += fixp(E, wsc) - fixp(En, wsc);
                    E = En;
                    if (!inside(S, rx, ry, rz)) {
                        l_esc += fixp(E, wsc);
                        record(P, h, (float)e0, n, hj, 2, (float)rx, (float)ry, (float)rz,
                               (float)E, j1, j2);
                        state = kDead;
                    } else if (E < S.e_min) {
                        score(P, S, tile, rep, acc, rx, ry, rz, E, wsc, l_esc);
                        record(P, h, (float)e0, n, hj, 3, (float)rx, (float)ry, (float)rz,
                               (float)E, j1, j2);
                        state = kDead;
                    }
                }
            }
        }
        // ---------------- end-of-range steps, a batch at a time ----------------
        // A lane whose energy passed the end-of-range screen waits here, so
        // that the wave runs the FP64 residual-range step for several lanes
        // at once instead of once per lane.  A lane whose residual range
        // exceeds the step after all takes an ordinary step next.
        if (flags & kEor) {
            const unsigned long long ends = __ballot(state == kEnd);
            if (ends && ((int)__popcll(ends) >= P.jump_batch || __ballot(state == kStep) == 0ull)) {
                if (state == kEnd) {
                    const double rres = range_g64(P, mat, (double)E) / (double)rho;
                    if (rres <= P.sd.step) {
                        const R hr = (R)(0.5 * rres);
                        score(P, S, tile, rep, acc, M::fma(ox, hr, rx), M::fma(oy, hr, ry),
                              M::fma(oz, hr, rz), E, wsc, l_esc);
                        l_steps++;
                        const R fr = (R)rres;
                        record(P, h, (float)e0, n + 1, hj, 1, (float)M::fma(ox, fr, rx),
                               (float)M::fma(oy, fr, ry), (float)M::fma(oz, fr, rz), (float)E,
                               j1, j2);
                        state = kDead;
                    } else {
                        state = kStep;
                        end_checked = true;
                    }
                }
            }
        }
        if (state != kStep) continue;

        // ---------------- one step of Eq. (VSDE) ----------------
        if ((long long)n >= P.max_steps) {
            atomicAdd(&P.ledger[4], (unsigned long long)fixp(E, wsc));
            record(P, h, (float)e0, n, hj, 4, (float)rx, (float)ry, (float)rz, (float)E, j1, j2);
            state = kDead;
            continue;
        }
        const float4 mc = matc[mat];

        // End of range: residual range within one step, decided in FP64 in the
        // batch above; the FP32 screen E <= ec(material) is exact-safe (ec
        // bounds the energy whose range fits a step at the densest voxel of
        // that material).
        if ((flags & kEor) && E <= (R)mc.z && !end_checked) {
            state = kEnd;
            continue;
        }
        end_checked = false;

        const R lnE = M::lg(E);
        const R tl = (lnE - S.ln_e_lo) * S.inv_dln;
        const int li = lattice_interval(tl, P.n_e);
        const R lf = tl - (R)li;
        float4 ta, tb;
        if constexpr (!M::f64) {
            ta = tab[mat * P.n_e + li];
            tb = tab[mat * P.n_e + li + 1];
        }
        const uint4 w = philox((uint32_t)h, (uint32_t)(h >> 32), n, 0u, k0, k1);

        // Continuous loss, Eq. (bethbloch) with Bragg additivity; clamped
        // straggling, Eq. (energystraggling), B_n ~ N(0, Delta).
        R zoa, log_pre;
        if constexpr (M::f64) {
            zoa = P.mats64[mat].zoa;
            log_pre = P.mats64[mat].log_pre;
        } else {
            zoa = mc.x;
            log_pre = mc.y;
        }
        const R p2 = E * (E + R(2) * (R)kMp);
        const R g = E + (R)kMp;
        const R b2 = p2 * M::rcp(g * g);
        R s1 = R(0);
        if (flags & kLoss) {
            const R L = log_pre + M::lg(p2) - b2;
            s1 = rho * S.c_bethe * zoa * L * M::rcp(b2);
        }
        const R a = s1 * S.step;
        R X = R(0);
        if (flags & kStraggle) {
            const R gm = g * (R(1) / (R)kMp);
            const R var = rho * S.c_strag * zoa * gm * gm * (R(1) - R(0.5) * b2);
            const R zE = M::sq(R(-2) * M::lg(u_hi<R>(w.x))) * M::cosr(u_hi<R>(w.y));
            X = fmin(fmax(M::sq(var) * S.sqrt_step * zE, -a), a);
        }
        const R Ep = fmax(E - a + X, R(0));

        // Jump test: none with probability exp(-Delta sigma).  float: elastic
        // rate (Rutherford + Mott) = el_E2 / E^2 with el_E2 smooth in ln E,
        // inelastic rate linear on the lattice; double: the elastic rate from
        // its closed form at E.
        bool jumped = false;
        if (flags & (kElastic | kInelastic)) {
            R rate;
            if ((flags & kEcut) && (flags & kElastic)) {
                // the cut 2.5 sigma(E) at this step's medium and density
                const Cut<R> cut = energy_cut(S, ld_sig2z(P, S, tab, mat, rho, E, li, lf));
                R el, ne_rate;
                R nucl;
                if constexpr (M::f64) {
                    const MatDev64& md = P.mats64[mat];
                    el = md.c_ruth0 * (cut.T - 0.5);
                    if (md.c_mott != 0.0)
                        el += md.c_mott * mott_bracket(S, cut, S.eta_pre / ::sqrt(E));
                    const double2 ha = P.hot64[(size_t)mat * P.n_e + li];
                    const double2 hb = P.hot64[(size_t)mat * P.n_e + li + 1];
                    ne_rate = ::fma(lf, hb.x - ha.x, ha.x);
                    nucl = nuclear_sum(P, S, md, E, li, lf, cut);
                } else {
                    const MatDev& md = P.mats[mat];
                    el = md.c_ruth0 * (cut.T - 0.5f);
                    if (md.c_mott != 0.0f)
                        el += md.c_mott * mott_bracket(S, cut, S.eta_pre * M::rsq(E));
                    ne_rate = fmaf(lf, tb.z - ta.z, ta.z);
                    nucl = R(0);
                    if constexpr (kNuc) nucl = nuclear_sum(P, S, md, E, li, lf, cut);
                }
                rate = el / (E * E) + nucl + ((flags & kInelastic) ? ne_rate : R(0));
            } else if constexpr (M::f64) {
                const MatDev64& md = P.mats64[mat];
                const double2 ha = P.hot64[(size_t)mat * P.n_e + li];
                const double2 hb = P.hot64[(size_t)mat * P.n_e + li + 1];
                rate = R(0);
                if (flags & kElastic) {
                    R el = md.c_ruth;
                    if (md.c_mott != 0.0)
                        el += md.c_mott * mott_bracket(S, fixed_cut(S), S.eta_pre / ::sqrt(E));
                    rate += el / (E * E) + nuclear_sum(P, S, md, E, li, lf, fixed_cut(S));
                }
                if (flags & kInelastic) rate += ::fma(lf, hb.x - ha.x, ha.x);
            } else {
                const float el_e2 = fmaf(lf, tb.w - ta.w, ta.w);
                const float ne_rate = fmaf(lf, tb.z - ta.z, ta.z);
                rate = ((flags & kElastic) ? el_e2 * M::rcp(E * E) : 0.0f) +
                       ((flags & kInelastic) ? ne_rate : 0.0f);
            }
            const R lam = S.step * rho * rate;
            R pj;
            if constexpr (M::f64)
                pj = -::expm1(-lam);
            else
                pj = lam < 0.05f
                    ? lam * fmaf(-0.5f * lam, fmaf(-lam * (1.0f / 3.0f), fmaf(-0.25f, lam, 1.0f), 1.0f), 1.0f)
                    : 1.0f - __expf(-lam);
            jumped = u_lo<R>(w.x, w.y, w.z) < pj;
        }

        // Deposit E_n - E' at the step midpoint (pre-step direction), move.
        // Both R_n and, when in_next, R_{n+1} lie in the box, and so does the
        // midpoint: its inside test is needed only when R_{n+1} left.
        const R nx = M::fma(ox, S.step, rx), ny = M::fma(oy, S.step, ry), nz = M::fma(oz, S.step, rz);
        const bool in_next = inside(S, nx, ny, nz);
        score(P, S, tile, rep, acc, M::fma(ox, S.half_step, rx), M::fma(oy, S.half_step, ry),
              M::fma(oz, S.half_step, rz), E - Ep, wsc, l_esc, !in_next);
        rx = nx;
        ry = ny;
        rz = nz;
        uint2 pk_next = make_uint2(0u, 0u);
        int v_next = vcache;
        if (in_next) {   // prefetch the next voxel while the direction is updated
            int ix, iy, iz;
            voxel3(P, S, rx, ry, rz, ix, iy, iz);
            v_next = voxel_index(ix, iy, iz, P.nx, P.ny, P.nz);
            if (v_next != vcache) pk_next = P.vox[v_next];
        }

        // Small-angle diffusion over time t = sigma^2 Delta / z, sigma the
        // Lynch-Dahl width: the spherical Brownian motion law (switch kSbm;
        // the lineage count's normal is the sine partner of Z_E's
        // Box-Muller pair) or the geodesic Gaussian step of per-axis
        // variance t.
        if (flags & kMcs) {
            R sig2;
            if constexpr (M::f64) {
                sig2 = ld_time64(P.mats64[mat], S, rho, E);
            } else {
                const float A1 = fmaf(lf, tb.x - ta.x, ta.x);
                const float A2 = fmaf(lf, tb.y - ta.y, ta.y);
                const float nu = rho * A2;
                const float br = (1.0f + M::rcp(nu)) * M::lg(1.0f + nu) - 1.0f;
                sig2 = rho * A1 * br;
            }
            R ct = R(1), st = R(0);
            bool now = true;
            if (flags & kSbm) {
                if (sig2 < SbmSwitch<R>::t) {
                    const R zM = M::sq(R(-2) * M::lg(u_hi<R>(w.x))) * M::sinr(u_hi<R>(w.y));
                    sbm_small(sig2, zM, u_hi<R>(w.z), ct, st);
                } else {   // exact regime: drawn at the top of the loop
                    now = false;
                    sbm_pend = true;
                    sbm_t = sig2;
                    sbm_u = u_hi<R>(w.z);
                    sbm_ph = u_hi<R>(w.w);
                }
            } else {
                polar_cs(R(-2) * sig2 * M::lg(u_hi<R>(w.z)), ct, st);
            }
            if (now) {
                const R ph = u_hi<R>(w.w);
                turn(ox, oy, oz, ct, st, M::cosr(ph), M::sinr(ph));
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
            const R inv = M::rsq(ox * ox + oy * oy + oz * oz);
            ox *= inv;
            oy *= inv;
            oz *= inv;
            E = Ep;
            n++;
            // Lane guard, folded into the exit test: a non-finite energy or
            // direction (one non-finite component reaches all three through
            // the renormalisation, and the move then leaves the box, so this
            // step's deposit was scored as escaped) ends the history; its
            // energy goes to the bad-lane ledger slot, so the energy balance
            // still closes, and its record ends with code 6.
            const bool bad = !__builtin_isfinite(E * ox);
            if (!in_next || bad) {
                if (bad) {
                    l_bad += __builtin_isfinite(E) ? fixp(E, wsc) : 0ll;
                    record(P, h, (float)e0, n, hj, 6, (float)rx, (float)ry, (float)rz, (float)E,
                           j1, j2);
                } else {
                    l_esc += fixp(E, wsc);
                    record(P, h, (float)e0, n, hj, 2, (float)rx, (float)ry, (float)rz, (float)E,
                           j1, j2);
                }
                state = kDead;
            } else if (E < S.e_min) {
                score(P, S, tile, rep, acc, rx, ry, rz, E, wsc, l_esc);
                record(P, h, (float)e0, n, hj, 3, (float)rx, (float)ry, (float)rz, (float)E, j1,
                       j2);
                state = kDead;
            }
        }
        if (in_next && v_next != vcache) {
            rho = (R)__uint_as_float(pk_next.x);
            mat = (int)pk_next.y;
            vcache = v_next;
        }
    }

    acc_flush(tile, rep, acc);
    // ledger: wave sums, one atomic per slot per wave
    const unsigned long long s_esc = wave_sum((unsigned long long)l_esc);
    const unsigned long long s_nuc = wave_sum((unsigned long long)l_nuc);
    const unsigned long long s_e0 = wave_sum((unsigned long long)l_e0);
    const unsigned long long s_st = wave_sum((unsigned long long)l_steps);
    const unsigned long long s_hi = wave_sum((unsigned long long)l_hist);
    const unsigned long long s_ju = wave_sum((unsigned long long)l_jumps);
    const unsigned long long s_bad = wave_sum((unsigned long long)l_bad);
    if (lane == 0) {
        if (s_bad) atomicAdd(&P.ledger[8], s_bad);
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
    if (t[i] < SbmSwitch<float>::t) {
        sbm_small(t[i], z[i], u[i], ct, st);
    } else {
        const CosSin<float> cs = sbm_large<float>((double)t[i], (double)u[i]);
        ct = cs.c;
        st = cs.s;
    }
    c[i] = ct;
    s[i] = st;
}

// Raw Philox4x32-10 blocks for given counters (the transport's generator),
// so that its words can be compared with another implementation bit for bit.
__global__ void k_philox_words(unsigned long long seed, const unsigned long long* __restrict__ h,
                               const unsigned* __restrict__ n, const unsigned* __restrict__ b,
                               int count, uint4* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const unsigned long long hh = h[i];
    out[i] = philox((uint32_t)hh, (uint32_t)(hh >> 32), n[i], b[i], (uint32_t)seed,
                    (uint32_t)(seed >> 32));
}

}  // namespace

hipError_t launch_philox_words(unsigned long long seed, const unsigned long long* h,
                               const unsigned* n, const unsigned* b, int count, uint4* out,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_philox_words, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       seed, h, n, b, count, out);
    return hipGetLastError();
}

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
    const void* fns[] = {reinterpret_cast<const void*>(&k_transport<float, kMethod, false>),
                         reinterpret_cast<const void*>(&k_transport<float, kMethodGeodesic, false>),
                         reinterpret_cast<const void*>(&k_transport<float, 0u, false>),
                         reinterpret_cast<const void*>(&k_transport<float, 0u, true>),
                         reinterpret_cast<const void*>(&k_transport<double, 0u, true>)};
    for (const void* f : fns) {
        const hipError_t e =
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_transport(const KParams& p, int grid, int block, size_t lds_bytes,
                            hipStream_t s) {
    if (p.fp64)
        hipLaunchKernelGGL((k_transport<double, 0u, true>), dim3(grid), dim3(block), lds_bytes, s,
                           p);
    else if (p.n_ni > 0 || p.n_l > 0)   // elastic nuclear data
        hipLaunchKernelGGL((k_transport<float, 0u, true>), dim3(grid), dim3(block), lds_bytes, s,
                           p);
    else if (p.flags == kMethod)
        hipLaunchKernelGGL((k_transport<float, kMethod, false>), dim3(grid), dim3(block),
                           lds_bytes, s, p);
    else if (p.flags == kMethodGeodesic)
        hipLaunchKernelGGL((k_transport<float, kMethodGeodesic, false>), dim3(grid), dim3(block),
                           lds_bytes, s, p);
    else
        hipLaunchKernelGGL((k_transport<float, 0u, false>), dim3(grid), dim3(block), lds_bytes, s,
                           p);
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

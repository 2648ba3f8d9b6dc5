// rt_physics.hpp -- per-lane arithmetic of the improved two-stream solve.
//
// Host- and device-callable so the same code can be unit-tested on a CPU.
// Paper: Deitrick et al., "The THOR+HELIOS general circulation model"
// (arXiv 2203.02293): Section 2.2.1 (layer relations, beam, boundary
// conditions, resonance guard), Section 2.2.4 (E fit), Appendix B
// (coefficients and source terms).  The coefficient forms used here are the
// paper's, rewritten without cancellation (see rt_kernels.hip).
#pragma once

#include <math.h>
#include <stdint.h>

#include "rt_internal.hpp"
#include "rt_math.hpp"

#include <limits>

namespace rtk {

constexpr double kPI = 3.141592653589793238462643383279502884;
constexpr double kH = 6.62607015e-34;   // SI 2019, exact
constexpr double kC = 299792458.0;
constexpr double kKB = 1.380649e-23;
constexpr double kPref = 2.0 * kKB * kKB * kKB * kKB / (kH * kH * kH * kC * kC);
constexpr double kPI4_15 = kPI * kPI * kPI * kPI / 15.0;

enum : uint32_t {
    F_GUARD = 1u, F_ECLAMP = 2u, F_ETAU = 4u, F_EDOMAIN = 8u, F_INVALID = 16u, F_NONFIN = 32u
};

// The condition bits of a column that fail a serving request (its status).
__host__ __device__ __forceinline__ uint32_t status_bits(uint32_t f)
{
    return f & (F_INVALID | F_EDOMAIN);
}

// ---------------------------------------------------------------------------
// Planck bin integrals.  With x = c2/(lambda T):
//   B_b(T) = (2 k^4 T^4 / (h^3 c^2)) * int_{x_a}^{x_b} t^3/(e^t - 1) dt.
// Small x: Q(x) = int_0^x = x^3/3 - x^4/8 + sum_k B_2k x^(2k+3)/((2k+3)(2k)!)
// (Bernoulli series, converges for x < 2 pi).  Large x: P(x) = int_x^inf =
// sum_n e^{-nx} (x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4).  Series coefficients are
// compile-time constants: B_2k/(2k)! = (-1)^{k+1} 2 zeta(2k)/(2 pi)^{2k}.
// ---------------------------------------------------------------------------
constexpr double zeta_even(int s)
{
    constexpr int M = 64;
    double sum = 0.0;
    for (int n = M - 1; n >= 1; --n) {
        double inv = 1.0 / n, t = 1.0;
        for (int i = 0; i < s; ++i) t *= inv;
        sum += t;
    }
    double Mi = 1.0 / M, Ms = 1.0, ds = s;
    for (int i = 0; i < s; ++i) Ms *= Mi;
    double tail = Ms * M / (ds - 1.0) + 0.5 * Ms + ds * Ms * Mi / 12.0
                - ds * (ds + 1) * (ds + 2) * Ms * Mi * Mi * Mi / 720.0
                + ds * (ds + 1) * (ds + 2) * (ds + 3) * (ds + 4) * Ms * Mi * Mi * Mi * Mi * Mi
                      / 30240.0;
    return sum + tail;
}

constexpr double bern_coef(int k)   // B_2k / ((2k+3) (2k)!)
{
    double tp = 1.0;
    for (int i = 0; i < 2 * k; ++i) tp *= 2.0 * kPI;
    double v = 2.0 * zeta_even(2 * k) / (tp * (2.0 * k + 3.0));
    return (k % 2 == 1) ? v : -v;
}

template <class R> struct PCfg;
template <> struct PCfg<double> {
    static constexpr double XS = 3.0;   // series switch
    static constexpr int NQ = 28;       // Bernoulli terms: (3/2pi)^56 < 1e-18
    static constexpr int NP = 13;       // exponential terms: e^-39 < 1e-16
    static constexpr double XCUT = 745.0;
};
template <> struct PCfg<float> {
    static constexpr float XS = 2.5f;
    static constexpr int NQ = 10;
    static constexpr int NP = 8;        // exponential terms: e^-20 < 2e-9
    static constexpr float XCUT = 104.0f;
};


constexpr double inv_factorial(int n)
{
    double f = 1.0;
    for (int m = 2; m <= n; ++m) f *= m;
    return 1.0 / f;
}

// coefficients 1/(2j+3)! of (sinh u - u)/u^3 as a series in u^2
struct SinhcCoef {
    static constexpr double coef(int j) { return inv_factorial(2 * j + 3); }
};
// coefficients c_k = B_2k/((2k+3)(2k)!) of the small-x Planck series, k >= 1
struct BernCoef {
    static constexpr double coef(int j) { return bern_coef(j + 1); }
};

// coefficients 1/n^S (n >= 1) of P_S(y) = sum_n y^n / n^S
template <int S>
struct InvPowCoef {
    static constexpr double coef(int j)
    {
        double v = 1.0;
        for (int i = 0; i < S; ++i) v /= double(j + 1);
        return v;
    }
};

// A set of lanes' largest need as a wavefront-uniform choice: whether any
// active lane of the wavefront has c true (every lane on the host).
__host__ __device__ __forceinline__ bool wave_any(bool c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_ballot_w64(c) != 0;
#else
    return c;
#endif
}

// FP64 large-x tail: sum_{n=1}^{M} e^{-nx} (x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4)
// = x^3 P_1(y) + 3x^2 P_2(y) + 6x P_3(y) + 6 P_4(y), y = e^{-x}, each P_S a
// Horner chain in y (four independent chains; z: an opaque zero, see horner_s).
template <int M>
__host__ __device__ __forceinline__ double planck_tail64(double x, double y, uint32_t z)
{
    const double p1 = y * horner_s<InvPowCoef<1>, 0, M>(y, z);
    const double p2 = y * horner_s<InvPowCoef<2>, 0, M>(y, z);
    const double p3 = y * horner_s<InvPowCoef<3>, 0, M>(y, z);
    const double p4 = y * horner_s<InvPowCoef<4>, 0, M>(y, z);
    return fma(x * x, fma(x, p1, 3.0 * p2), fma(6.0 * x, p3, 6.0 * p4));
}

// +Q(x) for x <= XS, -P(x) otherwise: the sign bit records which tail it is.
// x = c2/(lambda T) comes in FP64 in both precisions: FP32 takes e^-x from it
// with the low part of the argument applied (exp_em1_f).
// FP64: the number of series terms is the wavefront's largest need (a few
// fixed lengths, so every branch is uniform and every coefficient a
// compile-time constant): Q needs 15 terms up to x = 1.5 ((1.5/2pi)^30 <
// 1e-18) and 28 up to XS; P needs n terms while e^{-nx} is above 1e-17 of
// the first, i.e. n <= 39.1/x + 1, at most 13 above XS.
template <class R>
__host__ __device__ __forceinline__ R planck_edge(double xd)
{
    using Cfg = PCfg<R>;
    const R x = R(xd);
    if (x <= Cfg::XS) {
        const R x2 = x * x;
        R pb;
        if constexpr (sizeof(R) == 4) {
            pb = poly_eo<R, BernCoef, Cfg::NQ>(x2);
        } else {
            const uint32_t z = opaque_zero();
            if (wave_any(x > 1.5)) pb = horner_s<BernCoef, 0, Cfg::NQ>(x2, z);
            else pb = horner_s<BernCoef, 0, 15>(x2, z);
        }
        return x2 * x * (R(1.0 / 3.0) - R(0.125) * x + pb * x2);
    }
    if (!(x < Cfg::XCUT)) return R(-0.0);   // e^{-x} underflows (includes T = 0)
    // sum_{n>=1} y^n q_n, y = e^{-x}, q_n = x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4
    if constexpr (sizeof(R) == 4) {
        const R y = exp_em1_f(-xd).e;
        // FP32: forward from the largest term, over the terms that reach the
        // last bit: term n over term 1 is below y^(n-1) = e^-(n-1)x, under
        // 2^-25 once (n-1) x > 17.3.  The term index is the same in every lane
        // still summing, so the coefficients are constants; the wavefront
        // stops when its last lane has its terms (short-wave edges: one or two)
        const R x2 = x * x, x3 = x2 * x;
        const int nt = int(R(17.3) * rcp(x)) + 1;
        R yn = y, sum = R(0);
#pragma unroll
        for (int n = 1; n <= Cfg::NP; ++n) {
            if (n > nt) break;
            const double in = 1.0 / n;
            const R q = fma(x3, R(in), fma(x2, R(3 * in * in), fma(x, R(6 * in * in * in), R(6 * in * in * in * in))));
            sum = fma(yn, q, sum);
            yn *= y;
        }
        return -sum;
    } else {
        const R y = exp_em1(-x).e;
        const uint32_t z = opaque_zero();
        R sum;
        if (wave_any(x <= 39.1 / 8)) sum = planck_tail64<Cfg::NP>(x, y, z);
        else if (wave_any(x <= 39.1 / 4)) sum = planck_tail64<8>(x, y, z);
        else if (wave_any(x <= 39.1 / 2)) sum = planck_tail64<4>(x, y, z);
        else if (wave_any(x <= 39.1)) sum = planck_tail64<2>(x, y, z);
        else sum = planck_tail64<1>(x, y, z);
        return -sum;
    }
}

// int_{x_a}^{x_b} t^3/(e^t-1) dt from the two edge values (x_b > x_a):
// same tail on both sides: difference; straddling XS: pi^4/15 - P(x_b) - Q(x_a).
template <class R>
__host__ __device__ __forceinline__ R planck_combine(R vb, R va)
{
    R d = vb - va;
    if (signbit(vb) && !signbit(va)) d += R(kPI4_15);
    return d;
}

// int_{xa}^{xb} t^3/(e^t-1) dt by 3-point Gauss-Legendre in FP32: used for
// narrow bins, where the difference of two nearly equal edge integrals would
// lose digits.  The nodes are placed in FP64 and e^-x taken from them as in
// planck_edge.  The rule's relative error is below (xb-xa)^6 * 5e-7.
__host__ __device__ __forceinline__ float planck_gl3(double xa, double xb)
{
    const double h = 0.5 * (xb - xa), m = 0.5 * (xb + xa);
    const double d = 0.7745966692414834 * h;   // sqrt(3/5) h
    const double xs[3] = {m - d, m, m + d};
    const float ws[3] = {float(5.0 / 9.0), float(8.0 / 9.0), float(5.0 / 9.0)};
    float acc = 0.0f;
    for (int i = 0; i < 3; ++i) {
        const ExpEm1<float> e = exp_em1_f(-xs[i]);   // t^3 e^-t / (1 - e^-t)
        const float xf = float(xs[i]);
        acc += ws[i] * xf * xf * xf * e.e * rcp(-e.em1);
    }
    return float(h) * acc;
}

// Whether the FP32 difference of the two edge values of bin [xa, xb] would
// lose more than about 4 bits (edge value over bin integral above ~16), so
// that the bin takes the quadrature above instead.  Below XS both edges are
// integrals from 0 that grow like x^3/3, and the loss depends only on the
// bin's relative width: (xa/xb)^3 > 15/16.  Above XS (and across it) the edge
// values are at most pi^4/15 (large x: x^3 e^-x (1 + 3/x + ...)) against an
// integral of about (xb - xa) times the integrand: xb - xa <= 0.3 bounds the
// ratio by ~16.
template <class R>
__host__ __device__ __forceinline__ bool planck_narrow(R xa, R xb)
{
    if (xb > PCfg<R>::XS) return xb - xa <= R(0.3);
    return xa * xa * xa > R(0.9375) * (xb * xb * xb);
}

// ---------------------------------------------------------------------------
// Predicates in FP64, rounded exactly as the printed formulas read left to
// right (no contraction), so that both precisions take the paper's branch
// decisions on the same values.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ double efit_exact(double w0, double g0, const Opts &o, uint32_t &fl)
{
#pragma clang fp contract(off)
    if (!o.improved || !(w0 > 0.1)) return 1.0;
    double E = 1.225 - 0.1582 * g0 - 0.1777 * w0 - 0.07465 * g0 * g0
             + 0.2351 * w0 * g0 - 0.05582 * w0 * w0;
    if (o.e_clamp) {
        if (E < 1.0) {
            E = 1.0;
            fl |= F_ECLAMP;
        }
    } else if (E <= w0) {
        fl |= F_EDOMAIN;
    }
    return E;
}

__host__ __device__ __forceinline__ double resonance_D(double E, double w0, double g0, double mu)
{
#pragma clang fp contract(off)
    double ms = -mu;
    return 4.0 * E * ms * ms * (E - w0) * (1.0 - w0 * g0) - 1.0;
}

// ---------------------------------------------------------------------------
// helper functions of u
// ---------------------------------------------------------------------------
template <class R>
__host__ __device__ __forceinline__ R phi1(R x)   // (1 - e^-x)/x, x >= 0
{
    return (x > R(0)) ? -exp_em1(-x).em1 * rcp(x) : R(1);
}

template <class R> struct ShCfg;
template <> struct ShCfg<double> { static constexpr int N = 12; };
template <> struct ShCfg<float> { static constexpr int N = 7; };

// e^-u (sinh u - u)/u^2, u >= 0, given T = e^-u
template <class R>
__host__ __device__ __forceinline__ R hfun(R u, R T)
{
    if (u < R(2)) {
        // (sinh u - u)/u^2 = u sum_{k>=1} u^{2(k-1)} / (2k+1)!
        return T * u * poly<R, SinhcCoef, ShCfg<R>::N>(u * u);
    }
    return (R(0.5) * (R(1) - T * T) - u * T) * rcp(u * u);
}

// omt = 1 - t, formed without subtraction: with omr, the complements of t
// and r keep their relative precision where t or r is close to 1.
template <class R>
struct Layer {
    R t, r, omr, A, Sup, Sdn, omt;
};

// Coefficients and normalised sources of one layer (see the file header).
// Differences near 1 (1 - w0, E - w0, 1 - w0 g0) arrive already formed in
// FP64 by the caller: in FP32 they would lose up to ~2 digits for cloud layers.
// Fup and Flo are the direct beam at the layer's top and bottom interfaces.
// THIN: the beam-source differences f (1 - t beta) and f (beta - t) formed
// from exponentials of exponent sums and differences (three more exponentials
// per day layer) instead of from f, t and f beta, where, for a layer thin to
// the beam and to the diffuse flux, they are O(dtau) differences of O(1)
// values: in FP32 their rounding, accumulated over thousands of thin layers,
// reaches ~1e-5 of the fluxes.
template <class R, bool THIN = false>
__host__ __device__ __forceinline__ void layer_terms(R dtau, R w0, R g0, R E, R omw, R Ew, R om,
                                                     bool day, R mu, R inv_mu, R Dres,
                                                     bool guard, R Fup, R Flo, R Blo, R Bup,
                                                     bool iso, R inv_eps2, Layer<R> &L)
{
    const R one = R(1), half = R(0.5);
    const R Eom = E * om;
    R kap = R(2) * Eom;
    const R iEom = rcp(Eom);
    R ik = R(0.5) * iEom;   // 1/kappa
    // s = sqrt(Ew/Eom) and 1/s from one reciprocal square root (Ew = 0: s = 0;
    // Ew < 0, E below w0 in the unclamped fit: NaN, as sqrt gives)
    const R s2 = Ew * iEom;
    const bool spos = s2 > R(0);
    const R is = spos ? rsqrt_pos(s2) : (s2 == R(0) ? R(0) : std::numeric_limits<R>::quiet_NaN());
    R s = s2 * is;
    R lam = kap * s;
    R u = lam * dtau;
    ExpEm1<R> ex = exp_em1(-u);
    R Tr = ex.e, omT = -ex.em1;
    R zp = half * (one + s), zm = half * (one - s);
    R p = spos ? omT * is : kap * dtau;
    R q = p * (one + Tr);
    R den = fma(zm * zm, q, one);
    R id = rcp(den);
    R t = Tr * id;
    R r = zp * zm * q * id;
    R A = omT * (zp - zm * Tr) * id;
    L.t = t;
    L.omt = (omT + zm * zm * q) * id;   // (den - T) / den
    L.r = r;
    L.A = A;
    L.omr = (zp + zm * Tr * Tr) * id;
    R Pi = (E == one) ? R(kPI) : R(kPI) * omw * rcp(Ew);
    R Sup, Sdn;
    if (iso) {
        R Bm = half * (Blo + Bup);
        Sup = Pi * A * Bm;
        Sdn = Sup;
    } else {
        R ph = (u > R(0)) ? omT * rcp(u) : one;
        R Gd = u * (hfun(u, Tr) + half * s * ph * ph) * id;
        R dB = Blo - Bup;
        Sup = Pi * (A * Bup + dB * Gd);
        Sdn = Pi * (A * Blo - dB * Gd);
    }
    if (day) {
        R c1 = w0 * (kap + g0 * inv_eps2);
        R Qc = w0 * g0 * inv_eps2 * ik;
        R lm = lam * mu;
        R sb_up, sb_dn;
        // beta = e^-(dtau/mu), the layer's beam transmission, and 1 - beta from
        // one exponential (THIN: for every day layer; otherwise only near the
        // resonance).  Then 1 - beta T = (1 - beta) + beta (1 - T) has no
        // cancellation.
        R beta = R(0), omB = R(0);
        if constexpr (THIN) {
            const ExpEm1<R> eb = exp_em1(-dtau * inv_mu);
            beta = eb.e;
            omB = -eb.em1;
        }
        if (guard || fabs(lm - one) >= R(0.25)) {
            R Dd = guard ? R(-2) * mu : Dres;
            R P = c1 * rcp(Dd);
            R Gp = half * (P * (ik - mu) + Qc);
            R Gm = -half * (P * (ik + mu) + Qc);
            // f [r G- - G+ (1 - t beta)] and f [r beta G+ - G- (beta - t)], f beta = Flo
            if constexpr (THIN) {
                // 1 - t beta = (1 - T beta + zm^2 q) / den and
                // beta - t = (beta - T + beta zm^2 q) / den.  beta - T is
                // formed as (1 - T) - (1 - beta) for a layer thin to the beam
                // (beta >= 1/2) and directly otherwise: away from mu lambda = 1,
                // |lambda - 1/mu| >= 1/(4 mu), so either form loses at most a
                // factor of about 6 (under 3 bits) to cancellation
                const R zq = zm * zm * q;
                const R obt = omB + beta * omT;
                const R bmT = beta < half ? beta - Tr : omT - omB;
                sb_up = Fup * (r * Gm - Gp * (obt + zq) * id);
                sb_dn = r * Gp * Flo - Gm * Fup * (bmT + beta * zq) * id;
            } else {
                sb_up = r * Gm * Fup - Gp * (Fup - t * Flo);
                sb_dn = r * Gp * Flo - Gm * (Flo - t * Fup);
            }
        } else {
            // resonance-regularised: X, Yh = Y (a - lambda) are finite at mu lambda = 1
            R a = inv_mu;
            if constexpr (!THIN) {
                const ExpEm1<R> eb = exp_em1(-dtau * inv_mu);
                beta = eb.e;
                omB = -eb.em1;
            }
            R i1s = rcp(one + s);
            R X = (Qc - c1 * ik * rcp(one + lm)) * i1s;
            R Yh = (Qc * (a - lam) - c1 * a * ik) * i1s;
            R dq = (a >= lam) ? Tr * phi1((a - lam) * dtau) : beta * phi1((lam - a) * dtau);
            R Z = Yh * dq * dtau;
            R rho = zm * rcp(zp);
            R iom = (zp * zp) * rcp(s * den);       // 1 / (1 - rho^2 T^2)
            R obt = omB + beta * omT;               // 1 - beta T
            sb_up = Fup * (rho * Tr * Z - X * obt) * iom;
            sb_dn = Fup * (rho * Tr * X * obt - Z) * iom;
        }
        Sup += sb_up;
        Sdn += sb_dn;
    }
    L.Sup = Sup;
    L.Sdn = Sdn;
}

// Direct beam at an interface of optical depth tau below the TOA (Section
// 2.2.1, Beer's law), mu = -mu_star > 0.  The mixed path takes the
// exponential in FP32 of the FP64 argument tau/mu (exp_em1_f).
template <bool MIXED>
__host__ __device__ __forceinline__ double beam_at(double mu_Fstar, double tau, double inv_mu)
{
    if constexpr (MIXED) return mu_Fstar * double(exp_em1_f(-tau * inv_mu).e);
    else return mu_Fstar * exp_em1(-tau * inv_mu).e;
}

// Layer j between interfaces j and j+1 (Section 2.2.1, Appendix B): the
// paper's branch decisions in FP64, the coefficients in R.  Fb_up and Fb_lo
// are the beam at the top and bottom interfaces; Blo, Bup the Planck bin
// radiances there.
template <bool MIXED, class R, bool THIN = false>
__host__ __device__ __forceinline__ Layer<R> layer_item(double dt, double w, double g, bool day,
                                                        double mu, double inv_mu, double Fb_up,
                                                        double Fb_lo, R Blo, R Bup, const Opts &o,
                                                        double inv_eps2, uint32_t &fl)
{
    if (!(dt >= 0.0) || !isfinite(dt) || !(w >= 0.0 && w <= 1.0) || !(g > -1.0 && g < 1.0))
        fl |= F_INVALID;
    const double E = efit_exact(w, g, o, fl);
    bool guard = false;
    double D = 0.0;
    if (day) {
        D = resonance_D(E, w, g, mu);
        guard = fabs(D) < o.g_guard;
        if (guard) fl |= F_GUARD;
    }
    const bool iso = !o.noniso || dt < o.e_tau;
    if (o.noniso && dt < o.e_tau) fl |= F_ETAU;
    Layer<R> Ly;
    layer_terms<R, THIN>(R(dt), R(w), R(g), R(E), R(1.0 - w), R(E - w), R(1.0 - w * g), day, R(mu),
                   R(inv_mu), R(D), guard, R(Fb_up), R(Fb_lo), Blo, Bup, iso, R(inv_eps2), Ly);
    return Ly;
}

// ---------------------------------------------------------------------------
// Thomas elimination from the TOA (Section 2.2.2) on the normalised relations
//   F_up_{j+1} = t F_up_j + r F_dn_{j+1} + S_up,  F_dn_j = t F_dn_{j+1} + r F_up_j + S_dn.
// State at interface i: F_dn_i = c F_up_i + d, with eps = 1 - c carried
// without subtraction.  Always FP64.
// ---------------------------------------------------------------------------
struct ElimState {
    double c, eps, d;
};

// What the back-substitution needs of layer j: F_up_{j+1} = G F_up_j + H,
// F_dn_{j+1} = c F_up_{j+1} + d.
struct BackRec {
    double G, H, c, d;
};

__host__ __device__ __forceinline__ ElimState elim_top(double F_toa)
{
    ElimState s;
    s.c = 0.0;      // nothing above the TOA reflects
    s.eps = 1.0;
    s.d = F_toa;    // F_dn_N = F_TOA
    return s;
}

__host__ __device__ __forceinline__ BackRec elim_step(ElimState &st, double t, double r,
                                                      double omr, double A, double Sup,
                                                      double Sdn)
{
    const double inv = rcp(omr + r * st.eps);   // 1 / (1 - r c_{j+1})
    BackRec rec;
    rec.G = t * inv;
    rec.H = (r * st.d + Sup) * inv;
    rec.c = st.c;
    rec.d = st.d;
    const double cn = r + t * t * st.c * inv;
    const double en = (A * (omr + t) + st.eps * (r * omr + t * t)) * inv;
    const double dn = Sdn + t * (st.d + st.c * Sup) * inv;
    st.c = cn;
    st.eps = en;
    st.d = dn;
    return rec;
}

// BOA condition F_up_0 - F_dn_0 = F_BOA + F_beam_0 closes the elimination.
__host__ __device__ __forceinline__ void elim_boa(const ElimState &st, double F_boa, double Fb0,
                                                  double &Fu, double &Fd)
{
    Fu = (F_boa + Fb0 + st.d) / st.eps;
    Fd = st.c * Fu + st.d;
}

// One back-substitution step from interface j to j+1.
__host__ __device__ __forceinline__ void back_step(double G, double H, double c, double d,
                                                   double &Fu, double &Fd)
{
    Fu = G * Fu + H;
    Fd = c * Fu + d;
}

}  // namespace rtk

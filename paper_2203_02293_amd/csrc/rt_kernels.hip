// rt_kernels.hip -- gfx950 kernels of the improved two-stream solve.
//
// One lane owns one (column, bin).  Lanes are laid out bin-fastest, so each
// layer step of the sweep reads dtau/w0/g0 for a run of consecutive
// (column, bin) pairs: one coalesced load per array.  A workgroup holds K
// whole columns, which lets the Planck edge integrals of a column be computed
// once per interface and shared through LDS by all of its bins, and lets the
// bin sums be done in LDS in a fixed order.
//
// Paper: Deitrick et al., "The THOR+HELIOS general circulation model"
// (arXiv 2203.02293).  Section 2.2.1 (layer relations, beam, boundary
// conditions, resonance guard), Section 2.2.2 (Thomas algorithm), Section
// 2.2.4 (E fit), Appendix B (coefficients and source terms).
//
// The coefficients are the paper's, rewritten into forms without cancellation
// (all equalities are exact algebra, not approximations):
//   s = sqrt((E-w0)/(E(1-w0 g0))), zeta+- = (1 +- s)/2, kappa = 2E(1-w0 g0),
//   lambda = kappa s, u = lambda dtau, T = exp(-u),
//   t = psi/chi, r = -xi/chi   (normalised relations F_up_top = t F_up_bot + r F_dn_top + S_up)
//   with p = (1-T)/s (-> kappa dtau as s -> 0), q = p (1+T), den = 1 + zeta-^2 q:
//   t = T/den, r = zeta+ zeta- q/den, 1-r = (zeta+ + zeta- T^2)/den,
//   A = 1-r-t = (1-T)(zeta+ - zeta- T)/den  (layer absorptance, no subtraction),
//   thermal: S_up = Pi (A B_up + dB Gd), S_dn = Pi (A B_lo - dB Gd), dB = B_lo - B_up,
//   Gd = u [T (sinh u - u)/u^2 + (s/2) phi(u)^2] / den, phi(u) = (1 - e^-u)/u,
//   which equals (Theta/chi - t dtau)/dtau of Appendix B without its cancellation.
//   beam: away from the mu*lambda = 1 resonance the particular-solution form
//   S_up = f [r G- - G+ (1 - t beta)], S_dn = f [r beta G+ - G- (beta - t)]
//   (f = beam at the layer top, beta = exp(-dtau/mu), G+- with mu_star = -mu);
//   near it the same quantity regularised by dividing out (mu lambda - 1).
#include "rt_internal.hpp"

#include <math.h>
#include <type_traits>

namespace rtk {
namespace {

constexpr double kPI = 3.141592653589793238462643383279502884;
constexpr double kH = 6.62607015e-34;   // SI 2019, exact
constexpr double kC = 299792458.0;
constexpr double kKB = 1.380649e-23;
constexpr double kPref = 2.0 * kKB * kKB * kKB * kKB / (kH * kH * kH * kC * kC);
constexpr double kPI4_15 = kPI * kPI * kPI * kPI / 15.0;

enum : uint32_t {
    F_GUARD = 1u, F_ECLAMP = 2u, F_ETAU = 4u, F_EDOMAIN = 8u, F_INVALID = 16u, F_NONFIN = 32u
};

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
};
template <> struct PCfg<float> {
    static constexpr float XS = 2.5f;
    static constexpr int NQ = 10;
    static constexpr int NP = 8;
};

template <class R, int K, int NQ>
__device__ __forceinline__ R bern_horner(R x2)
{
    if constexpr (K == NQ) {
        return R(bern_coef(NQ));
    } else {
        return fma(bern_horner<R, K + 1, NQ>(x2), x2, R(bern_coef(K)));
    }
}

// +Q(x) for x <= XS, -P(x) otherwise: the sign bit records which tail it is.
template <class R>
__device__ __forceinline__ R planck_edge(R x)
{
    using Cfg = PCfg<R>;
    if (x <= Cfg::XS) {
        R x2 = x * x;
        R poly = bern_horner<R, 1, Cfg::NQ>(x2);
        return x2 * x * (R(1.0 / 3.0) - R(0.125) * x + poly * x2);
    }
    R y = exp(-x), yn = y, sum = R(0);
#pragma unroll
    for (int n = 1; n <= Cfg::NP; ++n) {
        const R in = R(1) / R(n);
        R poly = ((x * in + R(3) * in * in) * x + R(6) * in * in * in) * x
               + R(6) * in * in * in * in;
        sum = fma(yn, poly, sum);
        yn *= y;
    }
    return -sum;
}

// int_{x_a}^{x_b} t^3/(e^t-1) dt from the two edge values (x_b > x_a):
// same tail on both sides: difference; straddling XS: pi^4/15 - P(x_b) - Q(x_a).
template <class R>
__device__ __forceinline__ R planck_combine(R vb, R va)
{
    R d = vb - va;
    if (signbit(vb) && !signbit(va)) d += R(kPI4_15);
    return d;
}

// ---------------------------------------------------------------------------
// Predicates in FP64, rounded exactly as the printed formulas read left to
// right (no contraction), so that both precisions take the paper's branch
// decisions on the same values.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double efit_exact(double w0, double g0, const Opts &o, uint32_t &fl)
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

__device__ __forceinline__ double resonance_D(double E, double w0, double g0, double mu)
{
#pragma clang fp contract(off)
    double ms = -mu;
    return 4.0 * E * ms * ms * (E - w0) * (1.0 - w0 * g0) - 1.0;
}

// ---------------------------------------------------------------------------
// helper functions of u
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ R phi1(R x)   // (1 - e^-x)/x, x >= 0
{
    return (x > R(0)) ? -expm1(-x) / x : R(1);
}

template <class R> struct ShCfg;
template <> struct ShCfg<double> { static constexpr int N = 12; };
template <> struct ShCfg<float> { static constexpr int N = 7; };

// e^-u (sinh u - u)/u^2, u >= 0, given T = e^-u
template <class R>
__device__ __forceinline__ R hfun(R u, R T)
{
    if (u < R(2)) {
        // (sinh u - u)/u^2 = u sum_{k>=1} u^{2(k-1)} / (2k+1)!
        R u2 = u * u, acc = R(0);
#pragma unroll
        for (int k = ShCfg<R>::N; k >= 1; --k) {
            double f = 1.0;
            for (int m = 2; m <= 2 * k + 1; ++m) f *= m;
            acc = fma(acc, u2, R(1.0 / f));
        }
        return T * u * acc;
    }
    return (R(0.5) * (R(1) - T * T) - u * T) / (u * u);
}

template <class R>
struct Layer {
    R t, r, omr, A, Sup, Sdn;
};

// Coefficients and normalised sources of one layer (see the file header).
template <class R>
__device__ __forceinline__ void layer_terms(R dtau, R w0, R g0, R E, bool day, R mu, R Dres,
                                            bool guard, R f, R beta, R Blo, R Bup, bool iso,
                                            R eps2, Layer<R> &L)
{
    const R one = R(1), half = R(0.5);
    R om = one - w0 * g0;
    R Ew = E - w0;
    R kap = R(2) * E * om;
    R s = sqrt(Ew / (E * om));
    R lam = kap * s;
    R u = lam * dtau;
    R Tr = exp(-u);
    R omT = -expm1(-u);
    R zp = half * (one + s), zm = half * (one - s);
    R p = (s > R(0)) ? omT / s : kap * dtau;
    R q = p * (one + Tr);
    R den = fma(zm * zm, q, one);
    R id = one / den;
    R t = Tr * id;
    R r = zp * zm * q * id;
    R A = omT * (zp - zm * Tr) * id;
    L.t = t;
    L.r = r;
    L.A = A;
    L.omr = (zp + zm * Tr * Tr) * id;
    R Pi = (E == one) ? R(kPI) : R(kPI) * (one - w0) / Ew;
    R Sup, Sdn;
    if (iso) {
        R Bm = half * (Blo + Bup);
        Sup = Pi * A * Bm;
        Sdn = Sup;
    } else {
        R ph = (u > R(0)) ? omT / u : one;
        R Gd = u * (hfun(u, Tr) + half * s * ph * ph) * id;
        R dB = Blo - Bup;
        Sup = Pi * (A * Bup + dB * Gd);
        Sdn = Pi * (A * Blo - dB * Gd);
    }
    if (day) {
        R c1 = w0 * (kap + g0 / eps2);
        R Qc = w0 * g0 / (eps2 * kap);
        R lm = lam * mu;
        R sb_up, sb_dn;
        if (guard || fabs(lm - one) >= R(0.25)) {
            R Dd = guard ? R(-2) * mu : Dres;
            R P = c1 / Dd;
            R ik = one / kap;
            R Gp = half * (P * (ik - mu) + Qc);
            R Gm = -half * (P * (ik + mu) + Qc);
            sb_up = f * (r * Gm - Gp * (one - t * beta));
            sb_dn = f * (r * beta * Gp - Gm * (beta - t));
        } else {
            // resonance-regularised: X, Yh = Y (a - lambda) are finite at mu lambda = 1
            R a = one / mu;
            R X = (Qc - c1 / (kap * (one + lm))) / (one + s);
            R Yh = (Qc * (a - lam) - c1 * a / kap) / (one + s);
            R dq = (a >= lam) ? Tr * phi1((a - lam) * dtau) : beta * phi1((lam - a) * dtau);
            R Z = Yh * dq * dtau;
            R rho = zm / zp;
            R iom = (zp * zp) / (s * den);          // 1 / (1 - rho^2 T^2)
            R obt = -expm1(-(a + lam) * dtau);      // 1 - beta T
            sb_up = f * (rho * Tr * Z - X * obt) * iom;
            sb_dn = f * (rho * Tr * X * obt - Z) * iom;
        }
        Sup += sb_up;
        Sdn += sb_dn;
    }
    L.Sup = Sup;
    L.Sdn = Sdn;
}

// LDS chunk of interfaces reduced at once over bins
__host__ __device__ constexpr int lds_budget() { return 60 * 1024; }

__host__ __device__ inline int chunk_for(int threads, int K, int NB)
{
    int fixed = K * (NB + 1) * 8 + K * 9 * 8 + K * 4 + 64;
    int ch = (lds_budget() - fixed) / (3 * threads * 8);
    if (ch > 8) ch = 8;
    if (ch < 1) ch = 1;
    return ch;
}

// ---------------------------------------------------------------------------
// The solve kernel: Planck, coefficients, beam, forward elimination from the
// TOA, back-substitution from the BOA, bin sums, net flux and heating.
// ---------------------------------------------------------------------------
template <bool MIXED>
__global__ void __launch_bounds__(512) k_solve(const SolveArgs a)
{
    using R = typename std::conditional<MIXED, float, double>::type;
    extern __shared__ double smem[];
    const int NB = a.NB, K = a.K, C = a.C, N = a.N;
    const int tid = threadIdx.x, bd = blockDim.x;
    const int kloc = tid / NB, b = tid - kloc * NB;
    const int c = blockIdx.x * K + kloc;
    const bool active = (kloc < K) && (c < C);
    const long long gl = (long long)blockIdx.x * bd + tid;
    const int CH = chunk_for(bd, K, NB);
    const int nedge = K * (NB + 1);

    R *s_edge = reinterpret_cast<R *>(smem);                  // [K][NB+1]
    double *s_red = smem + nedge;                              // [3][CH][bd]
    double *s_fnet = s_red + 3 * CH * bd;                      // [K][CH+1]
    uint32_t *s_flag = reinterpret_cast<uint32_t *>(s_fnet + K * (CH + 1));  // [K]

    for (int kk = tid; kk < K; kk += bd) s_flag[kk] = 0u;
    uint32_t fl = 0u;

    // Planck radiance of this lane's bin at one level; all threads take part.
    auto planck_level = [&](const double *Tsrc, long long off) -> R {
        __syncthreads();
        for (int e = tid; e < nedge; e += bd) {
            int kk = e / (NB + 1), ee = e - kk * (NB + 1);
            int cc = blockIdx.x * K + kk;
            R v = R(0);
            if (cc < C) {
                double T = Tsrc[off + cc];
                R x;
                if constexpr (MIXED) x = a.c2_over_lam_f[ee] / float(T);
                else x = a.c2_over_lam[ee] / T;
                v = planck_edge<R>(x);
            }
            s_edge[e] = v;
        }
        __syncthreads();
        R B = R(0);
        if (active) {
            R T = R(Tsrc[off + c]);
            R T2 = T * T;
            B = R(kPref) * T2 * T2
              * planck_combine<R>(s_edge[kloc * (NB + 1) + b], s_edge[kloc * (NB + 1) + b + 1]);
        }
        return B;
    };

    double mu = 0.0;
    bool day = false;
    if (active) {
        mu = a.mu[c];
        day = mu > 0.0;
        if (!isfinite(mu)) fl |= F_INVALID;
        double ti = a.Tint[c];
        if (!(ti >= 0.0) || !isfinite(ti)) fl |= F_INVALID;
    }
    const double Fboa = double(kPI) * double(planck_level(a.Tint, 0));
    R Bup = planck_level(a.T, (long long)N * C);
    if (active) {
        double T = a.T[(long long)N * C + c];
        if (!(T > 0.0) || !isfinite(T)) fl |= F_INVALID;
    }

    double cc_ = 0.0, eps = 1.0, d = 0.0;
    double Fb = 0.0, tau = 0.0;
    R Fstar = R(0);
    if (active) {
        if (a.Ftoa) d = a.Ftoa[(long long)c * NB + b];
        if (day) {
            Fb = mu * a.F_star[b];
            Fstar = R(a.F_star[b]);
        }
    }
    const double inv_mu = day ? 1.0 / mu : 0.0;
    const long long LB = (long long)C * NB;
    const long long L = a.L;

    for (int j = N - 1; j >= 0; --j) {
        R Blo = planck_level(a.T, (long long)j * C);
        if (active) {
            const long long idx = (long long)j * LB + (long long)c * NB + b;
            const double dt = a.dtau[idx], w = a.w0[idx], g = a.g0[idx];
            const double Tl = a.T[(long long)j * C + c];
            if (!(dt >= 0.0) || !isfinite(dt) || !(w >= 0.0 && w <= 1.0) || !(g > -1.0 && g < 1.0)
                || !(Tl > 0.0) || !isfinite(Tl))
                fl |= F_INVALID;
            const double E = efit_exact(w, g, a.o, fl);
            bool guard = false;
            double D = 0.0;
            if (day) {
                D = resonance_D(E, w, g, mu);
                guard = fabs(D) < a.o.g_guard;
                if (guard) fl |= F_GUARD;
            }
            const bool iso = !a.o.noniso || dt < a.o.e_tau;
            if (a.o.noniso && dt < a.o.e_tau) fl |= F_ETAU;

            double Fb_lo = 0.0;
            R beta = R(0);
            if (day) {
                if constexpr (MIXED) {
                    tau += dt;
                    Fb_lo = mu * double(a.F_star[b]) * double(expf(float(-tau * inv_mu)));
                    beta = expf(float(-dt * inv_mu));
                } else {
                    beta = exp(-dt * inv_mu);
                    Fb_lo = Fb * beta;
                }
            }
            Layer<R> Ly;
            layer_terms<R>(R(dt), R(w), R(g), R(E), day, R(mu), R(D), guard, R(Fb), beta, Blo,
                           Bup, iso, R(a.o.eps2), Ly);
            const double t = Ly.t, r = Ly.r, omr = Ly.omr, A = Ly.A;
            const double Sup = Ly.Sup, Sdn = Ly.Sdn;
            // Thomas forward elimination (FP64): F_dn_i = c_i F_up_i + d_i,
            // eps_i = 1 - c_i carried without subtraction.
            const double inv = 1.0 / (omr + r * eps);
            double *sp = a.scratch + (long long)j * 5 * L + gl;
            sp[0] = t * inv;                  // G_j: F_up_{j+1} = G_j F_up_j + H_j
            sp[L] = (r * d + Sup) * inv;      // H_j
            sp[2 * L] = cc_;                  // c_{j+1}
            sp[3 * L] = d;                    // d_{j+1}
            sp[4 * L] = Fb;                   // beam at interface j+1
            const double cn = r + t * t * cc_ * inv;
            const double en = (A * (omr + t) + eps * (r * omr + t * t)) * inv;
            const double dn = Sdn + t * (d + cc_ * Sup) * inv;
            cc_ = cn;
            eps = en;
            d = dn;
            Fb = Fb_lo;
        }
        Bup = Blo;
    }

    // BOA condition: F_up_0 - F_dn_0 = F_BOA + F_beam_0, with F_dn_0 = c_0 F_up_0 + d_0
    double Fu = 0.0, Fd = 0.0, Fbi = 0.0;
    if (active) {
        Fu = (Fboa + Fb + d) / eps;
        Fd = cc_ * Fu + d;
        Fbi = Fb;
        if (fl) atomicOr(&s_flag[kloc], fl);
    }

    // back-substitution upward, bin sums in chunks of CH interfaces
    for (int i0 = 0; i0 <= N; i0 += CH) {
        const int nch = min(CH, N + 1 - i0);
        for (int ii = 0; ii < nch; ++ii) {
            const int i = i0 + ii;
            if (active) {
                if (i > 0) {
                    const double *sp = a.scratch + (long long)(i - 1) * 5 * L + gl;
                    Fu = sp[0] * Fu + sp[L];
                    Fd = sp[2 * L] * Fu + sp[3 * L];
                    Fbi = sp[4 * L];
                }
                const long long k = ((long long)i * C + c) * NB + b;
                if (a.F_up_bin) a.F_up_bin[k] = Fu;
                if (a.F_dn_bin) a.F_dn_bin[k] = Fd;
                if (i == N && a.F_up_toa_bin) a.F_up_toa_bin[(long long)c * NB + b] = Fu;
            }
            s_red[(0 * CH + ii) * bd + tid] = active ? Fu : 0.0;
            s_red[(1 * CH + ii) * bd + tid] = active ? Fd : 0.0;
            s_red[(2 * CH + ii) * bd + tid] = active ? Fbi : 0.0;
        }
        __syncthreads();
        // bin sums: one task per (column, interface) of the chunk
        for (int task = tid; task < K * CH; task += bd) {
            const int kk = task / CH, ii = task - kk * CH;
            const int cc = blockIdx.x * K + kk;
            if (ii >= nch || cc >= C) continue;
            double su = 0.0, sd = 0.0, sb = 0.0;
            const double *ru = s_red + (0 * CH + ii) * bd + kk * NB;
            const double *rd = s_red + (1 * CH + ii) * bd + kk * NB;
            const double *rb = s_red + (2 * CH + ii) * bd + kk * NB;
            for (int bb = 0; bb < NB; ++bb) {
                su += ru[bb];
                sd += rd[bb];
                sb += rb[bb];
            }
            const long long o = (long long)(i0 + ii) * C + cc;
            const double fn = su - sd - sb;
            a.F_up[o] = su;
            a.F_dn[o] = sd;
            a.F_beam[o] = sb;
            a.F_net[o] = fn;
            s_fnet[kk * (CH + 1) + ii + 1] = fn;
            if (!isfinite(fn)) atomicOr(&s_flag[kk], F_NONFIN);
        }
        __syncthreads();
        // heating of the layer below each interface of the chunk
        for (int task = tid; task < K * CH; task += bd) {
            const int kk = task / CH, ii = task - kk * CH;
            const int cc = blockIdx.x * K + kk;
            const int i = i0 + ii;
            if (ii >= nch || cc >= C || i < 1) continue;
            const double dp = a.p[(long long)(i - 1) * C + cc] - a.p[(long long)i * C + cc];
            if (!(dp > 0.0)) atomicOr(&s_flag[kk], F_INVALID);
            const double qh =
                a.o.gravity * (s_fnet[kk * (CH + 1) + ii] - s_fnet[kk * (CH + 1) + ii + 1]) / dp;
            a.heat[(long long)(i - 1) * C + cc] = qh;
            if (a.dTdt) a.dTdt[(long long)(i - 1) * C + cc] = qh / a.o.cp;
        }
        __syncthreads();
        for (int kk = tid; kk < K; kk += bd) s_fnet[kk * (CH + 1)] = s_fnet[kk * (CH + 1) + nch];
        __syncthreads();
    }
    __syncthreads();
    for (int kk = tid; kk < K; kk += bd) {
        const int cc = blockIdx.x * K + kk;
        if (cc < C && a.flags) a.flags[cc] = s_flag[kk];
    }
}

}  // namespace

Geometry solve_geometry(int C, int NB)
{
    Geometry g;
    g.K = 256 / NB;
    if (g.K < 1) g.K = 1;
    if (g.K > C) g.K = C;
    int lanes = g.K * NB;
    g.threads = ((lanes + 63) / 64) * 64;
    g.blocks = (C + g.K - 1) / g.K;
    g.lanes = (long long)g.blocks * g.threads;
    const int ch = chunk_for(g.threads, g.K, NB);
    g.lds = (size_t)g.K * (NB + 1) * 8 + (size_t)3 * ch * g.threads * 8
          + (size_t)g.K * (ch + 1) * 8 + (size_t)g.K * 4;
    return g;
}

size_t solve_scratch_bytes(int C, int N, int NB)
{
    Geometry g = solve_geometry(C, NB);
    return (size_t)N * 5 * (size_t)g.lanes * sizeof(double);
}

hipError_t launch_solve(const SolveArgs &a, int precision, hipStream_t s)
{
    Geometry g = solve_geometry(a.C, a.NB);
    SolveArgs b = a;
    b.K = g.K;
    b.L = g.lanes;
    if (precision == 1)
        hipLaunchKernelGGL(k_solve<true>, dim3(g.blocks), dim3(g.threads), g.lds, s, b);
    else
        hipLaunchKernelGGL(k_solve<false>, dim3(g.blocks), dim3(g.threads), g.lds, s, b);
    return hipGetLastError();
}

}  // namespace rtk

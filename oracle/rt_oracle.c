/*
 * rt_oracle.c -- plain FP64 CPU oracle of the improved two-stream flux solve.
 *
 * TEST INFRASTRUCTURE ONLY (see rt_oracle.h).  It is written for a reader
 * holding the paper: every quantity is computed from its printed definition,
 * in FP64, one (column, bin) at a time, with no blocking, fusion or algebraic
 * rearrangement.  Paper: Deitrick et al., "The THOR+HELIOS general
 * circulation model" (arXiv 2203.02293).
 *
 *   Planck bin integral ........ Section 2.2.1 (B at interfaces), Eq. for F_BOA
 *   E(w0, g0) .................. Section 2.2.4, the generalised E fit
 *   zeta, T, chi, xi, psi, Pi .. Appendix B, coefficient equations and Pi
 *   G+- and the resonance guard  Appendix B (G factors), Section 2.2.1 (mu_crit)
 *   layer relations ............ Section 2.2.1 (isothermal / non-isothermal
 *                                flux relations), Appendix B (blackbody terms)
 *   boundary conditions ........ Section 2.2.1 (BOA condition), Fig. 5 caption
 *   block Thomas ............... Section 2.2.2
 *   net flux ................... Section 2.2.1: the beam is added to the
 *                                downward flux before the net flux is formed
 *
 * Readings where the paper is silent or ambiguous (each one is listed with
 * its reason in the project's design notes):
 *   - G+- use mu_star = -mu (negative zenith cosine, Appendix B convention);
 *   - guard: if |D| < g_guard then D := 2 mu_star;
 *   - e_clamp: E := max(E_fit, 1) where the fit applies; strict mode flags E <= w0;
 *   - isothermal layers use B = (B_lower + B_upper)/2;
 *   - one slab per layer, B linear in tau between its interface values;
 *   - Planck per bin is the integral of B_lambda over the bin (W m^-2 sr^-1);
 *   - heating Q_j = g (Fnet_j - Fnet_{j+1}) / (p_j - p_{j+1}).
 */
#include "rt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/*
 * Arithmetic type.  The oracle is FP64 (ORC_QUAD undefined).  The same source
 * compiled with -DORC_QUAD=1 evaluates every step in IEEE binary128
 * (__float128, libquadmath); that build measures the rounding error of FP64
 * evaluations of the printed formulas, which cancel badly for thin layers and
 * near the G+- resonance, and serves as the reference of the parity tests.
 */
#ifdef ORC_QUAD
#include <quadmath.h>
typedef __float128 real;
#define RF(f) f##q
#define K_(x) x##Q
#else
typedef double real;
#define RF(f) f
#define K_(x) x
#endif

#define ORC_PI K_(3.14159265358979323846264338327950288)
/* SI 2019 exact constants */
#define ORC_H K_(6.62607015e-34)
#define ORC_C K_(299792458.0)
#define ORC_K K_(1.380649e-23)

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes on [-1, 1] by Newton's method on P_n (textbook).     */
/* ------------------------------------------------------------------------ */
#define ORC_GL_N 20
static real gl_x[ORC_GL_N], gl_w[ORC_GL_N];
static int gl_ready = 0;

static void orc_gauss_legendre(void)
{
    const int n = ORC_GL_N;
    for (int i = 0; i < n; ++i) {
        real z = RF(cos)(ORC_PI * (i + K_(0.75)) / (n + K_(0.5))), dp = 0;
        for (int it = 0; it < 100; ++it) {
            real p0 = 1, p1 = 0;
            for (int k = 1; k <= n; ++k) {
                real p2 = p1;
                p1 = p0;
                p0 = ((2 * (real)k - 1) * z * p1 - ((real)k - 1) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1);
            real dz = p0 / dp;
            z -= dz;
            if (RF(fabs)(dz) < K_(1e-32)) break;
        }
        gl_x[i] = z;
        gl_w[i] = 2 / ((1 - z * z) * dp * dp);
    }
    gl_ready = 1;
}

/* integrand of the Planck bin integral in x = h c / (lambda k T) */
static real orc_planck_x(real x)
{
    if (x > 700) return 0;
    return x * x * x / RF(expm1)(x);
}

/*
 * Bin-integrated Planck radiance (W m^-2 sr^-1):
 *   B_b(T) = int_{lam1}^{lam2} 2 h c^2 / lam^5 / (exp(h c / (lam k T)) - 1) dlam
 * written with x = h c / (lam k T) as (2 k^4 T^4 / (h^3 c^2)) int x^3/(e^x-1) dx
 * and evaluated by composite 20-point Gauss-Legendre on panels of width <= 1.
 */
static real orc_planck_bin_r(real T, real lam1, real lam2)
{
    if (!gl_ready) orc_gauss_legendre();
    if (!(T > 0)) return 0;
    real xa = ORC_H * ORC_C / (lam2 * ORC_K * T);   /* long-wave edge  */
    real xb = ORC_H * ORC_C / (lam1 * ORC_K * T);   /* short-wave edge */
    if (xa > 700) return 0;
    if (xb > 750) xb = 750;
    int panels = (int)RF(ceil)(xb - xa);
    if (panels < 1) panels = 1;
    real h = (xb - xa) / panels, sum = 0;
    for (int p = 0; p < panels; ++p) {
        real a = xa + p * h, mid = a + h / 2, s = 0;
        for (int i = 0; i < ORC_GL_N; ++i)
            s += gl_w[i] * orc_planck_x(mid + h / 2 * gl_x[i]);
        sum += h / 2 * s;
    }
    real kT = ORC_K * T;
    real pref = 2 * kT * kT * kT * kT / (ORC_H * ORC_H * ORC_H * ORC_C * ORC_C);
    return pref * sum;
}

double orc_planck_bin(double T, double lam1, double lam2)
{
    return (double)orc_planck_bin_r(T, lam1, lam2);
}

/*
 * Ratio of first Eddington coefficients, Section 2.2.4.  The branch decisions
 * (w0 > 0.1, E_fit < 1, E <= w0) are always taken on the FP64 values, so the
 * extended build follows exactly the branches of the FP64 definition.
 */
static double orc_efit_double(double w0, double g0)
{
    return 1.225 - 0.1582 * g0 - 0.1777 * w0 - 0.07465 * g0 * g0
         + 0.2351 * w0 * g0 - 0.05582 * w0 * w0;
}

static real orc_efit_r(double w0, double g0, const orc_opts *o, uint32_t *flags)
{
    if (!o->improved || !(w0 > 0.1)) return 1;
    double Ed = orc_efit_double(w0, g0);
    real E = K_(1.225) - K_(0.1582) * g0 - K_(0.1777) * w0 - K_(0.07465) * g0 * g0
           + K_(0.2351) * w0 * g0 - K_(0.05582) * w0 * w0;
    if (o->e_clamp) {
        if (Ed < 1.0) { E = 1; *flags |= ORC_F_ECLAMP; }
    } else if (Ed <= w0) {
        *flags |= ORC_F_EDOMAIN;
    }
    return E;
}

double orc_efit(double w0, double g0, const orc_opts *o, uint32_t *flags)
{
    return (double)orc_efit_r(w0, g0, o, flags);
}

typedef struct { real E, zp, zm, Tr, chi, xi, psi, Pi, Gp, Gm, D; uint32_t flags; } lyr;

/*
 * Appendix B: coupling coefficients, transmission, chi/xi/psi, Pi and G+-.
 * The resonance guard decides on D evaluated in FP64 (see orc_efit_r).
 */
static void orc_layer_r(double dtau_d, double w0_d, double g0_d, double mu_d,
                        const orc_opts *o, lyr *L)
{
    memset(L, 0, sizeof(*L));
    real dtau = dtau_d, w0 = w0_d, g0 = g0_d, mu = mu_d;
    real E = orc_efit_r(w0_d, g0_d, o, &L->flags);
    real zp = (1 + RF(sqrt)((E - w0) / (E * (1 - w0 * g0)))) / 2;
    real zm = (1 - RF(sqrt)((E - w0) / (E * (1 - w0 * g0)))) / 2;
    real Tr = RF(exp)(-2 * RF(sqrt)(E * (E - w0) * (1 - w0 * g0)) * dtau);
    L->E = E;
    L->zp = zp;
    L->zm = zm;
    L->Tr = Tr;
    L->chi = zm * zm * Tr * Tr - zp * zp;
    L->xi = zp * zm * (1 - Tr * Tr);
    L->psi = (zm * zm - zp * zp) * Tr;
    L->Pi = ORC_PI * (1 - w0) / (E - w0);
    if (mu > 0) {
        real ms = -mu;   /* paper's negative zenith cosine */
        real D = 4 * E * ms * ms * (E - w0) * (1 - w0 * g0) - 1;
        double Ed = (double)E, msd = -mu_d;
        double Dd = 4.0 * Ed * msd * msd * (Ed - w0_d) * (1.0 - w0_d * g0_d) - 1.0;
        if (fabs(Dd) < o->g_guard) {
            D = 2 * ms;
            L->flags |= ORC_F_GUARD;
        }
        L->D = D;
        real eps2 = o->eps2;
        real a = w0 * (2 * E * (1 - w0 * g0) + g0 / eps2) / D;
        real b = 1 / (2 * E * (1 - w0 * g0));
        real c = w0 * g0 / (2 * eps2 * E * (1 - w0 * g0));
        L->Gp = (a * (ms + b) + c) / 2;
        L->Gm = (a * (ms - b) - c) / 2;
    }
}

void orc_layer_coeffs(double dtau, double w0, double g0, double mu,
                      const orc_opts *o, orc_layer *out)
{
    lyr L;
    orc_layer_r(dtau, w0, g0, mu, o, &L);
    out->E = L.E; out->zp = L.zp; out->zm = L.zm; out->Tr = L.Tr;
    out->chi = L.chi; out->xi = L.xi; out->psi = L.psi; out->Pi = L.Pi;
    out->Gp = L.Gp; out->Gm = L.Gm; out->D = L.D; out->flags = L.flags;
}

/*
 * Assemble the block-tridiagonal system A_i X_{i-1} + B_i X_i + C_i X_{i+1} = D_i
 * (Section 2.2.2) for one (column, bin).  X_i = (F_up_i, F_dn_i), i = 0..N.
 * Block row 0:         [BOA condition ; downward relation of layer 0]
 * Block row i (0<i<N): [upward relation of layer i-1 ; downward relation of layer i]
 * Block row N:         [upward relation of layer N-1 ; F_dn_N = F_toa]
 * Arrays A, Bm, Cm are [N+1][2][2] row-major, D is [N+1][2]; B[N+1] holds the
 * Planck values at the interfaces (index 0 = BOA).
 */
static void orc_assemble_r(int N, const real *B, const double *dtau, const double *w0,
                           const double *g0, long stride, real mu, real Fstar,
                           real F_boa, real F_toa, const orc_opts *o,
                           real *A, real *Bm, real *Cm, real *D, real *F_beam,
                           uint32_t *flags)
{
    for (long k = 0; k < 4L * (N + 1); ++k) A[k] = Bm[k] = Cm[k] = 0;
    for (long k = 0; k < 2L * (N + 1); ++k) D[k] = 0;

    /* direct beam, Beer's law from the top: tau_N = 0 */
    real tau = 0;
    F_beam[N] = (mu > 0) ? mu * Fstar : 0;
    for (int j = N - 1; j >= 0; --j) {
        tau += dtau[(long)j * stride];
        F_beam[j] = (mu > 0) ? mu * Fstar * RF(exp)(-tau / mu) : 0;
    }

    /* BOA: F_up_0 - F_dn_0 = F_BOA + F_beam_0 */
    Bm[0] = 1;
    Bm[1] = -1;
    D[0] = F_boa + F_beam[0];
    /* TOA: F_dn_N = F_TOA */
    Bm[4 * N + 2] = 0;
    Bm[4 * N + 3] = 1;
    D[2 * N + 1] = F_toa;

    for (int j = 0; j < N; ++j) {
        double dt_d = dtau[(long)j * stride];
        real dt = dt_d;
        real w = w0[(long)j * stride], g = g0[(long)j * stride];
        lyr L;
        orc_layer_r(dt_d, w0[(long)j * stride], g0[(long)j * stride], (double)mu, o, &L);
        *flags |= L.flags;
        real Blo = B[j], Bup = B[j + 1], Bp = 0, Theta = 0;
        if (!o->noniso || dt_d < o->e_tau) {
            /* constant Planck function within the layer */
            if (o->noniso) *flags |= ORC_F_ETAU;
            Blo = Bup = (B[j] + B[j + 1]) / 2;
        } else {
            Bp = (B[j] - B[j + 1]) / dt;   /* dB/dtau, tau pointing down */
            Theta = (L.chi - L.psi - L.xi) / (2 * L.E * (1 - w * g));
        }
        real Fb_lo = F_beam[j], Fb_up = F_beam[j + 1];
        /* upward relation: chi F_up_{j+1} = psi F_up_j - xi F_dn_{j+1} + sources */
        real src_up = L.Pi * (Bup * (L.chi + L.xi) - L.psi * Blo + Bp * Theta)
                    + L.psi * L.Gp * Fb_lo - (L.xi * L.Gm + L.chi * L.Gp) * Fb_up;
        /* downward relation: chi F_dn_j = psi F_dn_{j+1} - xi F_up_j + sources */
        real src_dn = L.Pi * (Blo * (L.chi + L.xi) - L.psi * Bup - Bp * Theta)
                    + L.psi * L.Gm * Fb_up - (L.xi * L.Gp + L.chi * L.Gm) * Fb_lo;

        /* upward relation of layer j sits in row 0 of block row j+1 */
        int r = j + 1;
        A[4 * r + 0] = -L.psi;        /* coefficient of F_up_j     */
        Bm[4 * r + 0] = L.chi;        /* coefficient of F_up_{j+1} */
        Bm[4 * r + 1] = L.xi;         /* coefficient of F_dn_{j+1} */
        D[2 * r + 0] = src_up;
        /* downward relation of layer j sits in row 1 of block row j */
        Bm[4 * j + 2] = L.xi;         /* coefficient of F_up_j     */
        Bm[4 * j + 3] = L.chi;        /* coefficient of F_dn_j     */
        Cm[4 * j + 3] = -L.psi;       /* coefficient of F_dn_{j+1} */
        D[2 * j + 1] = src_dn;
    }
}

/* 2x2 helpers (row-major) */
static int inv2(const real *m, real *r)
{
    real det = m[0] * m[3] - m[1] * m[2];
    if (det == 0) return -1;
    r[0] = m[3] / det;
    r[1] = -m[1] / det;
    r[2] = -m[2] / det;
    r[3] = m[0] / det;
    return 0;
}
static void mul22(const real *a, const real *b, real *r)
{
    real t0 = a[0] * b[0] + a[1] * b[2], t1 = a[0] * b[1] + a[1] * b[3];
    real t2 = a[2] * b[0] + a[3] * b[2], t3 = a[2] * b[1] + a[3] * b[3];
    r[0] = t0; r[1] = t1; r[2] = t2; r[3] = t3;
}
static void mul21(const real *a, const real *v, real *r)
{
    real t0 = a[0] * v[0] + a[1] * v[1], t1 = a[2] * v[0] + a[3] * v[1];
    r[0] = t0; r[1] = t1;
}

/*
 * Block Thomas algorithm, Section 2.2.2:
 *   C'_0 = B_0^{-1} C_0,  D'_0 = B_0^{-1} D_0,
 *   C'_i = (B_i - A_i C'_{i-1})^{-1} C_i,
 *   D'_i = (B_i - A_i C'_{i-1})^{-1} (D_i - A_i D'_{i-1}),
 *   X_N = D'_N,  X_i = D'_i - C'_i X_{i+1}.
 */
static int orc_block_thomas_r(int N, const real *A, const real *Bm, const real *Cm,
                              const real *D, real *X)
{
    real *Cp = (real *)malloc(sizeof(real) * 4 * (N + 1));
    real *Dp = (real *)malloc(sizeof(real) * 2 * (N + 1));
    if (!Cp || !Dp) { free(Cp); free(Dp); return -2; }
    int rc = 0;
    for (int i = 0; i <= N && rc == 0; ++i) {
        real M[4], Minv[4], rhs[2], t[4], v[2];
        memcpy(M, Bm + 4 * i, sizeof(M));
        rhs[0] = D[2 * i];
        rhs[1] = D[2 * i + 1];
        if (i > 0) {
            mul22(A + 4 * i, Cp + 4 * (i - 1), t);
            for (int k = 0; k < 4; ++k) M[k] -= t[k];
            mul21(A + 4 * i, Dp + 2 * (i - 1), v);
            rhs[0] -= v[0];
            rhs[1] -= v[1];
        }
        if (inv2(M, Minv)) { rc = -1; break; }
        mul22(Minv, Cm + 4 * i, Cp + 4 * i);
        mul21(Minv, rhs, Dp + 2 * i);
    }
    if (rc == 0) {
        X[2 * N] = Dp[2 * N];
        X[2 * N + 1] = Dp[2 * N + 1];
        for (int i = N - 1; i >= 0; --i) {
            real v[2];
            mul21(Cp + 4 * i, X + 2 * (i + 1), v);
            X[2 * i] = Dp[2 * i] - v[0];
            X[2 * i + 1] = Dp[2 * i + 1] - v[1];
        }
    }
    free(Cp);
    free(Dp);
    return rc;
}

/* public wrappers of the assembly and the Thomas solver (double arrays) */
int orc_assemble(int N, const double *B, const double *dtau, const double *w0,
                 const double *g0, long stride, double mu, double Fstar,
                 double F_boa, double F_toa, const orc_opts *o,
                 double *A, double *Bm, double *Cm, double *D,
                 double *F_beam, uint32_t *flags)
{
    size_t n4 = 4 * (size_t)(N + 1), n2 = 2 * (size_t)(N + 1);
    real *buf = (real *)malloc(sizeof(real) * (3 * n4 + 2 * n2 + (N + 1)));
    if (!buf) return -2;
    real *rA = buf, *rB = rA + n4, *rC = rB + n4, *rD = rC + n4, *rF = rD + n2,
         *Br = rF + n2;
    for (int i = 0; i <= N; ++i) Br[i] = B[i];
    orc_assemble_r(N, Br, dtau, w0, g0, stride, mu, Fstar, F_boa, F_toa, o,
                   rA, rB, rC, rD, rF, flags);
    for (size_t k = 0; k < n4; ++k) { A[k] = rA[k]; Bm[k] = rB[k]; Cm[k] = rC[k]; }
    for (size_t k = 0; k < n2; ++k) D[k] = rD[k];
    for (int i = 0; i <= N; ++i) F_beam[i] = rF[i];
    free(buf);
    return 0;
}

int orc_block_thomas(int N, const double *A, const double *Bm, const double *Cm,
                     const double *D, double *X)
{
    size_t n4 = 4 * (size_t)(N + 1), n2 = 2 * (size_t)(N + 1);
    real *buf = (real *)malloc(sizeof(real) * (3 * n4 + 2 * n2));
    if (!buf) return -2;
    real *rA = buf, *rB = rA + n4, *rC = rB + n4, *rD = rC + n4, *rX = rD + n2;
    for (size_t k = 0; k < n4; ++k) { rA[k] = A[k]; rB[k] = Bm[k]; rC[k] = Cm[k]; }
    for (size_t k = 0; k < n2; ++k) rD[k] = D[k];
    int rc = orc_block_thomas_r(N, rA, rB, rC, rD, rX);
    for (size_t k = 0; k < n2; ++k) X[k] = rX[k];
    free(buf);
    return rc;
}

/* One (column, bin): assemble and solve; fluxes at the N+1 interfaces. */
static int orc_column_bin_r(int N, const real *B, const double *dtau, const double *w0,
                            const double *g0, long stride, real mu, real Fstar,
                            real F_boa, real F_toa, const orc_opts *o,
                            real *F_up, real *F_dn, real *F_beam, uint32_t *flags)
{
    size_t n4 = 4 * (size_t)(N + 1), n2 = 2 * (size_t)(N + 1);
    real *buf = (real *)malloc(sizeof(real) * (3 * n4 + 2 * n2));
    if (!buf) return -2;
    real *A = buf, *Bm = A + n4, *Cm = Bm + n4, *D = Cm + n4, *X = D + n2;
    orc_assemble_r(N, B, dtau, w0, g0, stride, mu, Fstar, F_boa, F_toa, o,
                   A, Bm, Cm, D, F_beam, flags);
    int rc = orc_block_thomas_r(N, A, Bm, Cm, D, X);
    for (int i = 0; i <= N; ++i) {
        F_up[i] = X[2 * i];
        F_dn[i] = X[2 * i + 1];
    }
    free(buf);
    return rc;
}

int orc_column_bin(int N, const double *B, const double *dtau, const double *w0,
                   const double *g0, long stride, double mu, double Fstar,
                   double F_boa, double F_toa, const orc_opts *o,
                   double *F_up, double *F_dn, double *F_beam, uint32_t *flags)
{
    real *buf = (real *)malloc(sizeof(real) * 4 * (N + 1));
    if (!buf) return -2;
    real *Br = buf, *fu = Br + (N + 1), *fd = fu + (N + 1), *fb = fd + (N + 1);
    for (int i = 0; i <= N; ++i) Br[i] = B[i];
    int rc = orc_column_bin_r(N, Br, dtau, w0, g0, stride, mu, Fstar, F_boa, F_toa, o,
                              fu, fd, fb, flags);
    for (int i = 0; i <= N; ++i) { F_up[i] = fu[i]; F_dn[i] = fd[i]; F_beam[i] = fb[i]; }
    free(buf);
    return rc;
}

static int orc_valid_column(const orc_problem *P, int c)
{
    const int C = P->n_cols, N = P->n_layers, NB = P->n_bins * P->n_gauss;
    if (!isfinite(P->mu_star[c]) || !(P->T_int[c] >= 0.0)) return 0;
    for (int i = 0; i <= N; ++i) {
        double T = P->T_iface[(long)i * C + c], p = P->p_iface[(long)i * C + c];
        if (!(T > 0.0) || !isfinite(T) || !(p > 0.0) || !isfinite(p)) return 0;
        if (i > 0 && !(P->p_iface[(long)(i - 1) * C + c] > p)) return 0;
    }
    for (int j = 0; j < N; ++j)
        for (int b = 0; b < NB; ++b) {
            long k = ((long)j * C + c) * NB + b;
            double dt = P->dtau[k], w = P->w0[k], g = P->g0[k];
            if (!(dt >= 0.0) || !isfinite(dt)) return 0;
            if (!(w >= 0.0 && w <= 1.0)) return 0;
            if (!(g > -1.0 && g < 1.0)) return 0;
        }
    return 1;
}

/* Whole problem: every (column, bin), bin sums, net flux and heating rate. */
int orc_solve(const orc_problem *P, const orc_opts *o, int n_threads)
{
    const int C = P->n_cols, N = P->n_layers, NB = P->n_bins, NG = P->n_gauss;
    const int NBG = NB * NG;   /* (bin, g-point) pairs per column */
    const int c0 = P->col_begin, c1 = P->col_end;
    if (C <= 0 || N <= 0 || NB <= 0 || NG <= 0 || c0 < 0 || c1 > C || c0 > c1) return -1;
    if (NG > 1 && !P->gauss_w) return -1;
    if (!gl_ready) orc_gauss_legendre();
    int rc_all = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc_all)
#endif
    for (int c = c0; c < c1; ++c) {
        real *B = (real *)malloc(sizeof(real) * 7 * (N + 1));
        real *fu = B + (N + 1), *fd = fu + (N + 1), *fb = fd + (N + 1);
        real *su = fb + (N + 1), *sd = su + (N + 1), *sb = sd + (N + 1);
        real *fnet = (real *)malloc(sizeof(real) * (N + 1));
        for (int i = 0; i <= N; ++i) su[i] = sd[i] = sb[i] = 0;
        uint32_t fl = orc_valid_column(P, c) ? 0u : ORC_F_INVALID;
        const real mu = P->mu_star[c];
        for (int b = 0; b < NB; ++b) {
            const real l1 = P->lambda_edges[b], l2 = P->lambda_edges[b + 1];
            for (int i = 0; i <= N; ++i)
                B[i] = orc_planck_bin_r(P->T_iface[(long)i * C + c], l1, l2);
            real F_boa = ORC_PI * orc_planck_bin_r(P->T_int[c], l1, l2);
            real toa = 0;
            for (int g = 0; g < NG; ++g) {
                const real wg = NG > 1 ? (real)P->gauss_w[g] : 1;
                const int bg = b * NG + g;
                real F_toa = P->F_toa ? P->F_toa[(long)c * NBG + bg] : 0;
                long off = (long)c * NBG + bg, stride = (long)C * NBG;
                int rc = orc_column_bin_r(N, B, P->dtau + off, P->w0 + off, P->g0 + off, stride,
                                          mu, P->F_star[b], F_boa, F_toa, o, fu, fd, fb, &fl);
                if (rc) rc_all |= 1;
                for (int i = 0; i <= N; ++i) {
                    su[i] += wg * fu[i];
                    sd[i] += wg * fd[i];
                    sb[i] += wg * fb[i];
                    long k = ((long)i * C + c) * NBG + bg;
                    if (P->F_up_bin) P->F_up_bin[k] = fu[i];
                    if (P->F_dn_bin) P->F_dn_bin[k] = fd[i];
                    if (P->F_beam_bin) P->F_beam_bin[k] = fb[i];
                }
                toa += wg * fu[N];
            }
            if (P->F_up_toa_bin) P->F_up_toa_bin[(long)c * NB + b] = toa;
        }
        for (int i = 0; i <= N; ++i) {
            long k = (long)i * C + c;
            P->F_up[k] = su[i];
            P->F_dn[k] = sd[i];
            P->F_beam[k] = sb[i];
            /* the beam is added to the downward flux before the net flux is formed */
            fnet[i] = su[i] - sd[i] - sb[i];
            P->F_net[k] = fnet[i];
            if (!isfinite(P->F_net[k])) fl |= ORC_F_NONFIN;
        }
        for (int j = 0; j < N; ++j) {
            long k = (long)j * C + c;
            real dp = (real)P->p_iface[k] - (real)P->p_iface[k + C];
            real q = o->gravity * (fnet[j] - fnet[j + 1]) / dp;
            P->heating[k] = q;
            if (P->dTdt) P->dTdt[k] = q / o->cp;
        }
        if (P->flags) P->flags[c] = fl;
        free(B);
        free(fnet);
    }
    return rc_all ? -3 : 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ======================================================================
 * Optical properties of a layer (the step before the solve)
 * ====================================================================== */

/*
 * Rayleigh scattering cross section per molecule, Appendix C:
 *   sigma = 24 pi^3 / (n_ref^2 lam^4) ((n_r^2 - 1)/(n_r^2 + 2))^2 K_lam,
 * with K_lam = 1 and the printed refractivity fits (lam' = lam / 1 um).  The
 * printed constants are CGS (n_ref in cm^-3, lam in cm, sigma in cm^2); the
 * result is returned in m^2.
 */
static double orc_rayleigh_cgs(double lam_cm, double n_ref, double n_r)
{
    double r = (n_r * n_r - 1.0) / (n_r * n_r + 2.0);
    double l4 = lam_cm * lam_cm * lam_cm * lam_cm;
    const double pi = 3.14159265358979323846;
    return 24.0 * pi * pi * pi / (n_ref * n_ref * l4) * r * r;
}

double orc_rayleigh_h2(double lam_m)
{
    double lp = lam_m / 1e-6;
    double n_r = 1.358e-4 * (1.0 + 7.52e-3 / (lp * lp)) + 1.0;
    return 1e-4 * orc_rayleigh_cgs(lam_m * 100.0, 2.68678e19, n_r);
}

double orc_rayleigh_he(double lam_m)
{
    double lp = lam_m / 1e-6;
    double n_r = 1e-8 * (2283.0 + 1.8102e13 / (1.5342e10 - 1.0 / (lp * lp))) + 1.0;
    return 1e-4 * orc_rayleigh_cgs(lam_m * 100.0, 2.546899e19, n_r);
}

/*
 * Gas scattering cross section of a bin, x_h2 sigma_H2 + x_he sigma_He
 * averaged over the bin in wavenumber (the bins are equal in wavenumber and
 * the paper averages the gas scattering over each bin): composite 20-point
 * Gauss-Legendre on 16 panels.
 */
double orc_rayleigh_bin(double lam1, double lam2, double x_h2, double x_he)
{
    if (!gl_ready) orc_gauss_legendre();
    const double nu1 = 1.0 / lam2, nu2 = 1.0 / lam1;   /* lam1 < lam2 */
    const int panels = 16;
    const double h = (nu2 - nu1) / panels;
    double sum = 0.0;
    for (int p = 0; p < panels; ++p) {
        double mid = nu1 + (p + 0.5) * h, s = 0.0;
        for (int i = 0; i < ORC_GL_N; ++i) {
            double lam = 1.0 / (mid + 0.5 * h * (double)gl_x[i]);
            s += (double)gl_w[i] * (x_h2 * orc_rayleigh_h2(lam) + x_he * orc_rayleigh_he(lam));
        }
        sum += 0.5 * h * s;
    }
    return sum / (nu2 - nu1);
}

/* last index i with grid[i] <= x, clamped to [0, n-2]; x clamped to the grid */
static int orc_bracket(const double *grid, int n, double *x)
{
    if (*x < grid[0]) *x = grid[0];
    if (*x > grid[n - 1]) *x = grid[n - 1];
    int i = 0;
    while (i < n - 2 && grid[i + 1] <= *x) ++i;
    return i;
}

/*
 * Absorption opacity of (bin, g-point) bg at temperature T and pressure p:
 * the pre-mixed k-table interpolated bilinearly in T and log10 p, values
 * outside the table taken at its edge.
 */
double orc_kappa_interp(const orc_optab *tb, double T, double p, int bg)
{
    const int nbg = tb->n_bins * tb->n_gauss;
    double x = T, y = log10(p);
    int i = tb->n_temp > 1 ? orc_bracket(tb->temp, tb->n_temp, &x) : 0;
    int j = tb->n_press > 1 ? orc_bracket(tb->log10p, tb->n_press, &y) : 0;
    double t = tb->n_temp > 1 ? (x - tb->temp[i]) / (tb->temp[i + 1] - tb->temp[i]) : 0.0;
    double u = tb->n_press > 1 ? (y - tb->log10p[j]) / (tb->log10p[j + 1] - tb->log10p[j]) : 0.0;
    int i1 = tb->n_temp > 1 ? i + 1 : i, j1 = tb->n_press > 1 ? j + 1 : j;
#define KAP(jj, ii) tb->kappa[((long)(jj) * tb->n_temp + (ii)) * nbg + bg]
    return (1 - t) * (1 - u) * KAP(j, i) + t * (1 - u) * KAP(j, i1)
         + (1 - t) * u * KAP(j1, i) + t * u * KAP(j1, i1);
#undef KAP
}

/*
 * Extinction per unit mass, single-scattering albedo and asymmetry of gas
 * plus condensates at one point (Section 2.2.3): with cross sections per gas
 * molecule, extinction = sigma_scat,gas + kappa m + f (sigma_abs,cl +
 * sigma_scat,cl);  w0 = (sigma_scat,gas + f sigma_scat,cl) / extinction;
 * g0 = f sigma_scat,cl g0,cl / (sigma_scat,gas + f sigma_scat,cl).
 */
void orc_optics_point(const orc_optab *tb, double T, double p, int bg, double *kext,
                      double *w0, double *g0)
{
    const int b = bg / tb->n_gauss;
    const double kap = orc_kappa_interp(tb, T, p, bg);
    const double sg = tb->sigma_gas[b];
    const double sa = tb->cloud_abs ? tb->f_cloud * tb->cloud_abs[b] : 0.0;
    const double ss = tb->cloud_scat ? tb->f_cloud * tb->cloud_scat[b] : 0.0;
    const double ext = sg + kap * tb->m_mean + sa + ss;   /* per molecule */
    *kext = ext / tb->m_mean;                              /* per unit mass */
    *w0 = ext > 0 ? (sg + ss) / ext : 0.0;
    *g0 = (sg + ss) > 0 && tb->cloud_g0 ? ss * tb->cloud_g0[b] / (sg + ss) : 0.0;
}

/*
 * dtau, w0, g0 of every slab, [S][C][NB*NG].  sub = 0: one slab per layer,
 * properties at the layer centre, dtau = extinction (p_j - p_{j+1}) / g.
 * sub = 1: the sub-layer grid; properties at interfaces and centres, each
 * sub-layer taking the arithmetic mean of its two levels (Section 2.2.1),
 * dtau = mean extinction x the sub-layer's pressure thickness / g.
 */
int orc_optics(const orc_optab *tb, int C, int N, int sub, const double *T_iface,
               const double *p_iface, const double *T_center, const double *p_center,
               double *dtau, double *w0, double *g0)
{
    const int nbg = tb->n_bins * tb->n_gauss;
    if (C <= 0 || N <= 0 || nbg <= 0 || !T_center || !p_center) return -1;
    for (int c = 0; c < C; ++c)
        for (int bg = 0; bg < nbg; ++bg) {
            if (!sub) {
                for (int j = 0; j < N; ++j) {
                    double ke, w, g;
                    orc_optics_point(tb, T_center[(long)j * C + c], p_center[(long)j * C + c], bg,
                                     &ke, &w, &g);
                    long k = ((long)j * C + c) * nbg + bg;
                    double dp = p_iface[(long)j * C + c] - p_iface[(long)(j + 1) * C + c];
                    dtau[k] = ke * dp / tb->gravity;
                    w0[k] = w;
                    g0[k] = g;
                }
            } else {
                for (int s = 0; s < 2 * N; ++s) {
                    double T0, p0, T1, p1, ke0, w00, g00, ke1, w01, g01;
                    /* level s and s+1: even levels are interfaces, odd ones centres */
                    int l0 = s, l1 = s + 1;
                    T0 = (l0 & 1) ? T_center[(long)(l0 >> 1) * C + c] : T_iface[(long)(l0 >> 1) * C + c];
                    p0 = (l0 & 1) ? p_center[(long)(l0 >> 1) * C + c] : p_iface[(long)(l0 >> 1) * C + c];
                    T1 = (l1 & 1) ? T_center[(long)(l1 >> 1) * C + c] : T_iface[(long)(l1 >> 1) * C + c];
                    p1 = (l1 & 1) ? p_center[(long)(l1 >> 1) * C + c] : p_iface[(long)(l1 >> 1) * C + c];
                    orc_optics_point(tb, T0, p0, bg, &ke0, &w00, &g00);
                    orc_optics_point(tb, T1, p1, bg, &ke1, &w01, &g01);
                    long k = ((long)s * C + c) * nbg + bg;
                    dtau[k] = 0.5 * (ke0 + ke1) * (p0 - p1) / tb->gravity;
                    w0[k] = 0.5 * (w00 + w01);
                    g0[k] = 0.5 * (g00 + g01);
                }
            }
        }
    return 0;
}

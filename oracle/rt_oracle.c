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

#define ORC_PI 3.14159265358979323846
/* SI 2019 exact constants */
#define ORC_H 6.62607015e-34
#define ORC_C 299792458.0
#define ORC_K 1.380649e-23

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes on [-1, 1] by Newton's method on P_n (textbook).     */
/* ------------------------------------------------------------------------ */
#define ORC_GL_N 20
static double gl_x[ORC_GL_N], gl_w[ORC_GL_N];
static int gl_ready = 0;

static void orc_gauss_legendre(void)
{
    const int n = ORC_GL_N;
    for (int i = 0; i < n; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        gl_x[i] = z;
        gl_w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    gl_ready = 1;
}

/* integrand of the Planck bin integral in x = h c / (lambda k T) */
static double orc_planck_x(double x)
{
    if (x > 700.0) return 0.0;
    return x * x * x / expm1(x);
}

/*
 * Bin-integrated Planck radiance (W m^-2 sr^-1):
 *   B_b(T) = int_{lam1}^{lam2} 2 h c^2 / lam^5 / (exp(h c / (lam k T)) - 1) dlam
 * written with x = h c / (lam k T) as (2 k^4 T^4 / (h^3 c^2)) int x^3/(e^x-1) dx
 * and evaluated by composite 20-point Gauss-Legendre on panels of width <= 1.
 */
double orc_planck_bin(double T, double lam1, double lam2)
{
    if (!gl_ready) orc_gauss_legendre();
    if (!(T > 0.0)) return 0.0;
    double xa = ORC_H * ORC_C / (lam2 * ORC_K * T);   /* long-wave edge  */
    double xb = ORC_H * ORC_C / (lam1 * ORC_K * T);   /* short-wave edge */
    if (xa > 700.0) return 0.0;
    if (xb > 750.0) xb = 750.0;
    int panels = (int)ceil(xb - xa);
    if (panels < 1) panels = 1;
    double h = (xb - xa) / panels, sum = 0.0;
    for (int p = 0; p < panels; ++p) {
        double a = xa + p * h, mid = a + 0.5 * h, s = 0.0;
        for (int i = 0; i < ORC_GL_N; ++i)
            s += gl_w[i] * orc_planck_x(mid + 0.5 * h * gl_x[i]);
        sum += 0.5 * h * s;
    }
    double kT = ORC_K * T;
    double pref = 2.0 * kT * kT * kT * kT / (ORC_H * ORC_H * ORC_H * ORC_C * ORC_C);
    return pref * sum;
}

/* Ratio of first Eddington coefficients, Section 2.2.4. */
double orc_efit(double w0, double g0, const orc_opts *o, uint32_t *flags)
{
    if (!o->improved || !(w0 > 0.1)) return 1.0;
    double E = 1.225 - 0.1582 * g0 - 0.1777 * w0 - 0.07465 * g0 * g0
             + 0.2351 * w0 * g0 - 0.05582 * w0 * w0;
    if (o->e_clamp) {
        if (E < 1.0) { E = 1.0; *flags |= ORC_F_ECLAMP; }
    } else if (E <= w0) {
        *flags |= ORC_F_EDOMAIN;
    }
    return E;
}

/* Appendix B: coupling coefficients, transmission, chi/xi/psi, Pi and G+-. */
void orc_layer_coeffs(double dtau, double w0, double g0, double mu,
                      const orc_opts *o, orc_layer *L)
{
    memset(L, 0, sizeof(*L));
    double E = orc_efit(w0, g0, o, &L->flags);
    double zp = 0.5 * (1.0 + sqrt((E - w0) / (E * (1.0 - w0 * g0))));
    double zm = 0.5 * (1.0 - sqrt((E - w0) / (E * (1.0 - w0 * g0))));
    double Tr = exp(-2.0 * sqrt(E * (E - w0) * (1.0 - w0 * g0)) * dtau);
    L->E = E;
    L->zp = zp;
    L->zm = zm;
    L->Tr = Tr;
    L->chi = zm * zm * Tr * Tr - zp * zp;
    L->xi = zp * zm * (1.0 - Tr * Tr);
    L->psi = (zm * zm - zp * zp) * Tr;
    L->Pi = ORC_PI * (1.0 - w0) / (E - w0);
    if (mu > 0.0) {
        double ms = -mu;   /* paper's negative zenith cosine */
        double D = 4.0 * E * ms * ms * (E - w0) * (1.0 - w0 * g0) - 1.0;
        if (fabs(D) < o->g_guard) {
            D = 2.0 * ms;
            L->flags |= ORC_F_GUARD;
        }
        L->D = D;
        double a = w0 * (2.0 * E * (1.0 - w0 * g0) + g0 / o->eps2) / D;
        double b = 1.0 / (2.0 * E * (1.0 - w0 * g0));
        double c = w0 * g0 / (2.0 * o->eps2 * E * (1.0 - w0 * g0));
        L->Gp = 0.5 * (a * (ms + b) + c);
        L->Gm = 0.5 * (a * (ms - b) - c);
    }
}

/*
 * Assemble the block-tridiagonal system A_i X_{i-1} + B_i X_i + C_i X_{i+1} = D_i
 * (Section 2.2.2) for one (column, bin).  X_i = (F_up_i, F_dn_i), i = 0..N.
 * Block row 0:       [BOA condition ; downward relation of layer 0]
 * Block row i (0<i<N): [upward relation of layer i-1 ; downward relation of layer i]
 * Block row N:       [upward relation of layer N-1 ; F_dn_N = F_toa]
 * Arrays A, Bm, Cm are [N+1][2][2] row-major, D is [N+1][2]; B[N+1] holds the
 * Planck values at the interfaces (index 0 = BOA).
 */
int orc_assemble(int N, const double *B, const double *dtau, const double *w0,
                 const double *g0, long stride, double mu, double Fstar,
                 double F_boa, double F_toa, const orc_opts *o,
                 double *A, double *Bm, double *Cm, double *D,
                 double *F_beam, uint32_t *flags)
{
    memset(A, 0, sizeof(double) * 4 * (N + 1));
    memset(Bm, 0, sizeof(double) * 4 * (N + 1));
    memset(Cm, 0, sizeof(double) * 4 * (N + 1));
    memset(D, 0, sizeof(double) * 2 * (N + 1));

    /* direct beam, Beer's law from the top: tau_N = 0 */
    double tau = 0.0;
    F_beam[N] = (mu > 0.0) ? mu * Fstar : 0.0;
    for (int j = N - 1; j >= 0; --j) {
        tau += dtau[(long)j * stride];
        F_beam[j] = (mu > 0.0) ? mu * Fstar * exp(-tau / mu) : 0.0;
    }

    /* BOA: F_up_0 - F_dn_0 = F_BOA + F_beam_0 */
    Bm[0] = 1.0;
    Bm[1] = -1.0;
    D[0] = F_boa + F_beam[0];
    /* TOA: F_dn_N = F_TOA */
    Bm[4 * N + 2] = 0.0;
    Bm[4 * N + 3] = 1.0;
    D[2 * N + 1] = F_toa;

    for (int j = 0; j < N; ++j) {
        double dt = dtau[(long)j * stride];
        orc_layer L;
        orc_layer_coeffs(dt, w0[(long)j * stride], g0[(long)j * stride], mu, o, &L);
        *flags |= L.flags;
        double Blo = B[j], Bup = B[j + 1], Bp = 0.0, Theta = 0.0;
        if (!o->noniso || dt < o->e_tau) {
            /* constant Planck function within the layer */
            if (o->noniso) *flags |= ORC_F_ETAU;
            Blo = Bup = 0.5 * (B[j] + B[j + 1]);
        } else {
            Bp = (B[j] - B[j + 1]) / dt;   /* dB/dtau, tau pointing down */
            Theta = (L.chi - L.psi - L.xi)
                  / (2.0 * L.E * (1.0 - w0[(long)j * stride] * g0[(long)j * stride]));
        }
        double Fb_lo = F_beam[j], Fb_up = F_beam[j + 1];
        /* upward relation: chi F_up_{j+1} = psi F_up_j - xi F_dn_{j+1} + sources */
        double src_up = L.Pi * (Bup * (L.chi + L.xi) - L.psi * Blo + Bp * Theta)
                      + L.psi * L.Gp * Fb_lo - (L.xi * L.Gm + L.chi * L.Gp) * Fb_up;
        /* downward relation: chi F_dn_j = psi F_dn_{j+1} - xi F_up_j + sources */
        double src_dn = L.Pi * (Blo * (L.chi + L.xi) - L.psi * Bup - Bp * Theta)
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
    return 0;
}

/* 2x2 helpers (row-major) */
static int inv2(const double *m, double *r)
{
    double det = m[0] * m[3] - m[1] * m[2];
    if (det == 0.0) return -1;
    r[0] = m[3] / det;
    r[1] = -m[1] / det;
    r[2] = -m[2] / det;
    r[3] = m[0] / det;
    return 0;
}
static void mul22(const double *a, const double *b, double *r)
{
    double t0 = a[0] * b[0] + a[1] * b[2], t1 = a[0] * b[1] + a[1] * b[3];
    double t2 = a[2] * b[0] + a[3] * b[2], t3 = a[2] * b[1] + a[3] * b[3];
    r[0] = t0; r[1] = t1; r[2] = t2; r[3] = t3;
}
static void mul21(const double *a, const double *v, double *r)
{
    double t0 = a[0] * v[0] + a[1] * v[1], t1 = a[2] * v[0] + a[3] * v[1];
    r[0] = t0; r[1] = t1;
}

/*
 * Block Thomas algorithm, Section 2.2.2:
 *   C'_0 = B_0^{-1} C_0,  D'_0 = B_0^{-1} D_0,
 *   C'_i = (B_i - A_i C'_{i-1})^{-1} C_i,
 *   D'_i = (B_i - A_i C'_{i-1})^{-1} (D_i - A_i D'_{i-1}),
 *   X_N = D'_N,  X_i = D'_i - C'_i X_{i+1}.
 */
int orc_block_thomas(int N, const double *A, const double *Bm, const double *Cm,
                     const double *D, double *X)
{
    double *Cp = (double *)malloc(sizeof(double) * 4 * (N + 1));
    double *Dp = (double *)malloc(sizeof(double) * 2 * (N + 1));
    if (!Cp || !Dp) { free(Cp); free(Dp); return -2; }
    int rc = 0;
    for (int i = 0; i <= N && rc == 0; ++i) {
        double M[4], Minv[4], rhs[2], t[4], v[2];
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
            double v[2];
            mul21(Cp + 4 * i, X + 2 * (i + 1), v);
            X[2 * i] = Dp[2 * i] - v[0];
            X[2 * i + 1] = Dp[2 * i + 1] - v[1];
        }
    }
    free(Cp);
    free(Dp);
    return rc;
}

/* One (column, bin): assemble and solve; fluxes at the N+1 interfaces. */
int orc_column_bin(int N, const double *B, const double *dtau, const double *w0,
                   const double *g0, long stride, double mu, double Fstar,
                   double F_boa, double F_toa, const orc_opts *o,
                   double *F_up, double *F_dn, double *F_beam, uint32_t *flags)
{
    size_t n4 = 4 * (size_t)(N + 1), n2 = 2 * (size_t)(N + 1);
    double *buf = (double *)malloc(sizeof(double) * (3 * n4 + 2 * n2));
    if (!buf) return -2;
    double *A = buf, *Bm = A + n4, *Cm = Bm + n4, *D = Cm + n4, *X = D + n2;
    orc_assemble(N, B, dtau, w0, g0, stride, mu, Fstar, F_boa, F_toa, o,
                 A, Bm, Cm, D, F_beam, flags);
    int rc = orc_block_thomas(N, A, Bm, Cm, D, X);
    for (int i = 0; i <= N; ++i) {
        F_up[i] = X[2 * i];
        F_dn[i] = X[2 * i + 1];
    }
    free(buf);
    return rc;
}

static int orc_valid_column(const orc_problem *P, int c)
{
    const int C = P->n_cols, N = P->n_layers, NB = P->n_bins;
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
    const int C = P->n_cols, N = P->n_layers, NB = P->n_bins;
    const int c0 = P->col_begin, c1 = P->col_end;
    if (C <= 0 || N <= 0 || NB <= 0 || c0 < 0 || c1 > C || c0 > c1) return -1;
    if (!gl_ready) orc_gauss_legendre();
    int rc_all = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc_all)
#endif
    for (int c = c0; c < c1; ++c) {
        double *B = (double *)malloc(sizeof(double) * (N + 1));
        double *fu = (double *)malloc(sizeof(double) * 3 * (N + 1));
        double *su = (double *)calloc(3 * (size_t)(N + 1), sizeof(double));
        double *fd = fu + (N + 1), *fb = fd + (N + 1);
        double *sd = su + (N + 1), *sb = sd + (N + 1);
        uint32_t fl = orc_valid_column(P, c) ? 0u : ORC_F_INVALID;
        const double mu = P->mu_star[c];
        for (int b = 0; b < NB; ++b) {
            const double l1 = P->lambda_edges[b], l2 = P->lambda_edges[b + 1];
            for (int i = 0; i <= N; ++i)
                B[i] = orc_planck_bin(P->T_iface[(long)i * C + c], l1, l2);
            double F_boa = ORC_PI * orc_planck_bin(P->T_int[c], l1, l2);
            double F_toa = P->F_toa ? P->F_toa[(long)c * NB + b] : 0.0;
            long off = (long)c * NB + b, stride = (long)C * NB;
            int rc = orc_column_bin(N, B, P->dtau + off, P->w0 + off, P->g0 + off, stride,
                                    mu, P->F_star[b], F_boa, F_toa, o, fu, fd, fb, &fl);
            if (rc) rc_all |= 1;
            for (int i = 0; i <= N; ++i) {
                su[i] += fu[i];
                sd[i] += fd[i];
                sb[i] += fb[i];
                long k = ((long)i * C + c) * NB + b;
                if (P->F_up_bin) P->F_up_bin[k] = fu[i];
                if (P->F_dn_bin) P->F_dn_bin[k] = fd[i];
                if (P->F_beam_bin) P->F_beam_bin[k] = fb[i];
            }
            if (P->F_up_toa_bin) P->F_up_toa_bin[(long)c * NB + b] = fu[N];
        }
        for (int i = 0; i <= N; ++i) {
            long k = (long)i * C + c;
            P->F_up[k] = su[i];
            P->F_dn[k] = sd[i];
            P->F_beam[k] = sb[i];
            /* the beam is added to the downward flux before the net flux is formed */
            P->F_net[k] = su[i] - sd[i] - sb[i];
            if (!isfinite(P->F_net[k])) fl |= ORC_F_NONFIN;
        }
        for (int j = 0; j < N; ++j) {
            long k = (long)j * C + c;
            double dp = P->p_iface[k] - P->p_iface[k + C];
            double q = o->gravity * (P->F_net[k] - P->F_net[k + C]) / dp;
            P->heating[k] = q;
            if (P->dTdt) P->dTdt[k] = q / o->cp;
        }
        if (P->flags) P->flags[c] = fl;
        free(B);
        free(fu);
        free(su);
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

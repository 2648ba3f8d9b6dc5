/*
 * rt_oracle.h -- plain FP64 CPU oracle of the improved two-stream flux solve
 * (Deitrick et al., "The THOR+HELIOS general circulation model", Section 2.2
 * and Appendix B).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library; only
 * the test-suite, the smoke check and the benchmark's CPU-baseline leg load
 * it.  The GPU library neither includes this header nor links this code, and
 * this code includes nothing from the GPU library.
 *
 * Conventions (paper, Section 2.2.1 and Appendix B):
 *   interface i = 0 is the bottom of the atmosphere (BOA), i = N the top (TOA);
 *   layer j lies between interfaces j (lower) and j+1 (upper);
 *   optical depth grows downward, tau_N = 0, tau_i = sum_{j>=i} dtau_j;
 *   mu > 0 is the cosine of the stellar zenith angle (mu <= 0: no beam); the
 *   beam-coupling coefficients G+- are evaluated with the paper's negative
 *   zenith cosine, mu_star = -mu.
 */
#ifndef RT_ORACLE_H
#define RT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* per-column condition bits (same meaning as the GPU library's flags) */
#define ORC_F_GUARD    1u   /* G+- resonance guard replaced the denominator   */
#define ORC_F_ECLAMP   2u   /* E fit below 1 was raised to 1                  */
#define ORC_F_ETAU     4u   /* dtau < e_tau: gradient term dropped            */
#define ORC_F_EDOMAIN  8u   /* strict mode: E <= w0 (coefficients undefined)  */
#define ORC_F_INVALID 16u   /* input outside its documented domain            */
#define ORC_F_NONFIN  32u   /* a non-finite output was produced               */

typedef struct {
    int32_t improved;  /* 1: E from the fit of Section 2.2.4, 0: E = 1        */
    int32_t noniso;    /* 1: Planck linear in tau within a layer, 0: constant */
    int32_t e_clamp;   /* 1: E = max(E_fit, 1); 0: strict (flag E <= w0)      */
    int32_t pad_;
    double eps2;       /* second Eddington coefficient of the beam (2/3)      */
    double e_tau;      /* isothermal fallback threshold on dtau (1e-4)        */
    double g_guard;    /* |D| threshold of the G+- resonance guard (1e-5)     */
    double gravity;    /* m s^-2, heating-rate conversion (47)               */
    double cp;         /* J kg^-1 K^-1, dT/dt = Q / cp (12436)               */
} orc_opts;

typedef struct {
    double E, zp, zm, Tr, chi, xi, psi, Pi, Gp, Gm, D;
    uint32_t flags;
} orc_layer;

/*
 * k-distribution (Section 2.1.3): each bin b holds NG quadrature points
 * (g-points) with weights w_g summing to 1; a g-point is solved like a bin
 * of its own (its bin's Planck function and stellar flux) and bin sums are
 * sum_b sum_g w_g F.  Arrays over "(bin, g)" use index b*NG + g.  NG = 1
 * (weights NULL) is the plain per-bin problem.
 */
typedef struct {
    int32_t n_cols, n_layers, n_bins, col_begin, col_end; /* [col_begin,col_end) */
    int32_t n_gauss;              /* NG >= 1 g-points per bin          */
    int32_t pad_;
    const double *gauss_w;        /* [NG] weights, or NULL when NG = 1 */
    const double *lambda_edges;   /* [NB+1] m                          */
    const double *F_star;         /* [NB]   W m^-2 at normal incidence */
    const double *p_iface;        /* [N+1][C] Pa                       */
    const double *T_iface;        /* [N+1][C] K                        */
    const double *dtau, *w0, *g0; /* [N][C][NB*NG]                     */
    const double *mu_star;        /* [C]                               */
    const double *T_int;          /* [C]                               */
    const double *F_toa;          /* [C][NB*NG] or NULL                */
    /* outputs */
    double *F_up, *F_dn, *F_beam, *F_net;  /* [N+1][C] weighted bin sums */
    double *heating, *dTdt;                /* [N][C] (dTdt may be NULL) */
    double *F_up_toa_bin;                  /* [C][NB] weighted over g, or NULL */
    double *F_up_bin, *F_dn_bin, *F_beam_bin; /* [N+1][C][NB*NG] or NULL */
    uint32_t *flags;                       /* [C] or NULL */
} orc_problem;

double orc_planck_bin(double T, double lam1, double lam2);
double orc_efit(double w0, double g0, const orc_opts *o, uint32_t *flags);
void orc_layer_coeffs(double dtau, double w0, double g0, double mu,
                      const orc_opts *o, orc_layer *out);
int orc_assemble(int N, const double *B, const double *dtau, const double *w0,
                 const double *g0, long stride, double mu, double Fstar,
                 double F_boa, double F_toa, const orc_opts *o,
                 double *A, double *Bm, double *Cm, double *D,
                 double *F_beam, uint32_t *flags);
int orc_block_thomas(int N, const double *A, const double *Bm, const double *Cm,
                     const double *D, double *X);
int orc_column_bin(int N, const double *B, const double *dtau, const double *w0,
                   const double *g0, long stride, double mu, double Fstar,
                   double F_boa, double F_toa, const orc_opts *o,
                   double *F_up, double *F_dn, double *F_beam, uint32_t *flags);
int orc_solve(const orc_problem *P, const orc_opts *o, int n_threads);
int orc_max_threads(void);

/*
 * Optical properties (the step before the solve, Sections 2.1.3 and 2.2.3,
 * Appendix C): a pre-mixed k-table of absorption opacity per unit mass over
 * (T, log10 p), gas Rayleigh scattering and condensates mixed by number.
 */
typedef struct {
    int32_t n_temp, n_press, n_bins, n_gauss;
    const double *temp;         /* [n_temp] K, ascending                          */
    const double *log10p;       /* [n_press] log10(p / Pa), ascending             */
    const double *kappa;        /* [n_press][n_temp][NB*NG] m^2 kg^-1             */
    const double *sigma_gas;    /* [NB] gas scattering cross section, m^2/molecule */
    const double *cloud_abs;    /* [NB] condensate absorption cross section, m^2, or NULL */
    const double *cloud_scat;   /* [NB] condensate scattering cross section, m^2, or NULL */
    const double *cloud_g0;     /* [NB] condensate asymmetry, or NULL             */
    double f_cloud;             /* condensate-to-gas number ratio                 */
    double m_mean;              /* mean molecular mass, kg                        */
    double gravity;             /* m s^-2                                         */
} orc_optab;

double orc_rayleigh_h2(double lam_m);
double orc_rayleigh_he(double lam_m);
double orc_rayleigh_bin(double lam1, double lam2, double x_h2, double x_he);
double orc_kappa_interp(const orc_optab *tb, double T, double p, int bg);
void orc_optics_point(const orc_optab *tb, double T, double p, int bg, double *kext,
                      double *w0, double *g0);
int orc_optics(const orc_optab *tb, int C, int N, int sub, const double *T_iface,
               const double *p_iface, const double *T_center, const double *p_center,
               double *dtau, double *w0, double *g0);

#ifdef __cplusplus
}
#endif
#endif

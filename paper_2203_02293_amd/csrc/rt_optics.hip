// rt_optics.hip -- optical properties of the slabs: the step before the solve.
//
// Paper: Deitrick et al., "The THOR+HELIOS general circulation model"
// (arXiv 2203.02293): Section 2.1.3 (pre-mixed k-tables over temperature and
// log pressure, Gaussian points per bin), Section 2.2.3 (mixing of gas and
// condensate scattering into w0 and g0), Section 2.2.1 (sub-layer values are
// means of centre and interface values), Appendix C (Rayleigh cross
// sections of H2 and He).
//
// One wavefront per (slab, column) cell: the cell's k-table bracket (grid
// cell and interpolation weights in temperature and log pressure) is the same
// for all of the cell's outputs (bin x Gaussian point) and is found once, as
// wavefront-uniform values; the lanes then take the outputs 64 at a time, the
// point index fastest, so consecutive lanes read consecutive k-table entries
// of the same (T, p) cell and write consecutive outputs.  FP64 throughout.
#include "rt_internal.hpp"

#include <cmath>
#include <vector>

namespace rtk {
namespace {

__device__ __forceinline__ int bracket(const double *grid, int n, double &x)
{
    // last i with grid[i] <= x, in [0, n-2]; x held inside the grid
    if (x < grid[0]) x = grid[0];
    if (x > grid[n - 1]) x = grid[n - 1];
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (grid[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct Props {
    double kext, w0, g0;   // extinction per unit mass, albedo, asymmetry
};

// A (T, p) point's k-table cell: lower corner (i, j) and weights (t, u).
struct Cell {
    int i, j;
    double t, u;
};

__device__ __forceinline__ Cell cell_at(const OpticsArgs &a, double T, double p)
{
    double x = T, y = log10(p);
    Cell q;
    q.i = bracket(a.temp, a.nT, x);
    q.j = bracket(a.log10p, a.nP, y);
    q.t = (x - a.temp[q.i]) / (a.temp[q.i + 1] - a.temp[q.i]);
    q.u = (y - a.log10p[q.j]) / (a.log10p[q.j + 1] - a.log10p[q.j]);
    return q;
}

// Properties of output bg (bin b) in the k-table cell q: bilinear opacity, then
// the mixing of gas and condensate extinction and scattering.
__device__ __forceinline__ Props props_at(const OpticsArgs &a, const Cell &q, int bg, int b)
{
    const double t = q.t, u = q.u;
    const long long row = (long long)a.nT * a.NBG;
    const double *k0 = a.kappa + (long long)q.j * row + (long long)q.i * a.NBG + bg;
    const double k00 = k0[0], k10 = k0[a.NBG], k01 = k0[row], k11 = k0[row + a.NBG];
    const double kap = (1 - t) * (1 - u) * k00 + t * (1 - u) * k10 + (1 - t) * u * k01 + t * u * k11;
    const double sg = a.sig_gas[b], sa = a.sig_cl_abs[b], ss = a.sig_cl_scat[b];
    const double scat = sg + ss;
    const double ext = scat + kap * a.m_mean + sa;   // per gas molecule
    Props r;
    r.kext = ext / a.m_mean;
    r.w0 = ext > 0.0 ? scat / ext : 0.0;
    r.g0 = scat > 0.0 ? ss * a.g0_cl[b] / scat : 0.0;
    return r;
}

constexpr int kOpticsThreads = 64;

__device__ __forceinline__ void optics_cell(const OpticsArgs &a, const long long cell)
{
    const int s = (int)(cell / a.C), c = (int)(cell - (long long)s * a.C);
    // the cell's values: uniform across the wavefront
    Cell q0, q1;
    double dp;
    if (!a.sub) {
        q0 = cell_at(a, a.Tc[(long long)s * a.C + c], a.pc[(long long)s * a.C + c]);
        q1 = q0;
        dp = a.p[(long long)s * a.C + c] - a.p[(long long)(s + 1) * a.C + c];
    } else {
        // sub-layer s between levels s and s+1: even levels interfaces, odd ones centres
        auto lev = [&](int l, double &T, double &p) {
            const long long o = (long long)(l >> 1) * a.C + c;
            T = (l & 1) ? a.Tc[o] : a.T[o];
            p = (l & 1) ? a.pc[o] : a.p[o];
        };
        double T0, p0, T1, p1;
        lev(s, T0, p0);
        lev(s + 1, T1, p1);
        q0 = cell_at(a, T0, p0);
        q1 = cell_at(a, T1, p1);
        dp = p0 - p1;
    }
    for (int bg = threadIdx.x; bg < a.NBG; bg += kOpticsThreads) {
        const int b = bg / a.NG;
        Props P;
        if (!a.sub) {
            P = props_at(a, q0, bg, b);
        } else {
            const Props A = props_at(a, q0, bg, b), B = props_at(a, q1, bg, b);
            P.kext = 0.5 * (A.kext + B.kext);
            P.w0 = 0.5 * (A.w0 + B.w0);
            P.g0 = 0.5 * (A.g0 + B.g0);
        }
        const long long e = cell * a.NBG + bg;
        a.dtau[e] = P.kext * dp / a.gravity;
        a.w0[e] = P.w0;
        a.g0[e] = P.g0;
    }
}

__global__ void __launch_bounds__(kOpticsThreads) k_optics(const OpticsArgs a)
{
    // cell = s C + c, over a grid of rows of gridDim.x workgroups
    const long long cell = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    if (cell < (long long)a.S * a.C) optics_cell(a, cell);
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on the
// Legendre recurrence.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Rayleigh cross section per molecule (m^2) from the Lorentz-Lorenz form of
// Appendix C, evaluated in the printed CGS units.
double rayleigh_cgs_to_si(double lam_m, double n_ref_cm3, double n_r)
{
    const double lam_cm = lam_m * 100.0;
    const double ll = (n_r * n_r - 1.0) / (n_r * n_r + 2.0);
    const double pi3 = M_PI * M_PI * M_PI;
    return 1e-4 * 24.0 * pi3 / (n_ref_cm3 * n_ref_cm3 * lam_cm * lam_cm * lam_cm * lam_cm) * ll * ll;
}

double sigma_h2(double lam_m)
{
    const double l2 = (lam_m * 1e6) * (lam_m * 1e6);
    return rayleigh_cgs_to_si(lam_m, 2.68678e19, 1.0 + 1.358e-4 * (1.0 + 7.52e-3 / l2));
}

double sigma_he(double lam_m)
{
    const double l2 = (lam_m * 1e6) * (lam_m * 1e6);
    return rayleigh_cgs_to_si(lam_m, 2.546899e19,
                              1.0 + 1e-8 * (2283.0 + 1.8102e13 / (1.5342e10 - 1.0 / l2)));
}

}  // namespace

double rayleigh_bin_average(double lam_lo, double lam_hi, double x_h2, double x_he)
{
    // mean over the bin in wavenumber: 16 Gauss-Legendre points on 24 panels
    static std::vector<double> gx, gw;
    if (gx.empty()) gauss_legendre(16, gx, gw);
    const double nu0 = 1.0 / lam_hi, nu1 = 1.0 / lam_lo;
    const int panels = 24;
    const double h = (nu1 - nu0) / panels;
    double sum = 0.0;
    for (int pnl = 0; pnl < panels; ++pnl) {
        const double m = nu0 + (pnl + 0.5) * h;
        for (size_t i = 0; i < gx.size(); ++i) {
            const double lam = 1.0 / (m + 0.5 * h * gx[i]);
            sum += 0.5 * h * gw[i] * (x_h2 * sigma_h2(lam) + x_he * sigma_he(lam));
        }
    }
    return sum / (nu1 - nu0);
}

hipError_t launch_optics(const OpticsArgs &a, hipStream_t s)
{
    const long long cells = (long long)a.S * a.C;
    if (cells == 0 || a.NBG == 0) return hipSuccess;
    // one workgroup per cell: rows of up to 2^30 workgroups
    const long long row = cells < (1LL << 30) ? cells : (1LL << 30);
    const long long rows = (cells + row - 1) / row;
    hipLaunchKernelGGL(k_optics, dim3((unsigned)row, (unsigned)rows), dim3(kOpticsThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace rtk

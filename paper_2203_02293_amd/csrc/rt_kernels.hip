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
#include "rt_math.hpp"
#include "rt_physics.hpp"

#include <math.h>
#include <algorithm>
#include <type_traits>

namespace rtk {
namespace {

// LDS chunk of interfaces reduced at once over bins
__host__ __device__ constexpr int lds_budget() { return 60 * 1024; }

constexpr int PC = 8;   // levels whose Planck edges are computed per barrier

__host__ __device__ inline int chunk_for(int threads, int K, int NB)
{
    int fixed = K * 9 * 8 + K * 4 + 64;
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
__device__ __forceinline__ void solve_tile(const SolveArgs &a, const int tile)
{
    using R = typename std::conditional<MIXED, float, double>::type;
    extern __shared__ double smem[];
    const int NB = a.NB, K = a.K, C = a.C, N = a.N;
    const int tid = threadIdx.x, bd = blockDim.x;
    const int kloc = tid / NB, b = tid - kloc * NB;
    const int c = tile * K + kloc;
    const bool active = (kloc < K) && (c < C);
    const long long gl = (long long)tile * bd + tid;
    const int CH = chunk_for(bd, K, NB);

    // LDS: the forward sweep's Planck edge values and the back-substitution's
    // bin-sum buffers are live at different times and share the same bytes.
    R *s_pl = reinterpret_cast<R *>(smem);                     // [PC][K][NB+1]
    double *s_red = smem;                                      // [3][CH][bd]
    const int nslot = PC * K * (NB + 1);
    const int front = max(3 * CH * bd, nslot);
    double *s_fnet = smem + front;                             // [K][CH+1]
    uint32_t *s_flag = reinterpret_cast<uint32_t *>(s_fnet + K * (CH + 1));  // [K]

    for (int kk = tid; kk < K; kk += bd) s_flag[kk] = 0u;
    uint32_t fl = 0u;

    // Edge integrals of PC levels (rows q = 0..n-1 of level pointer src[q]) into LDS,
    // edge-major so that a wavefront's lanes mostly sit in one series regime.
    auto edge_chunk = [&](const double *Tsrc, long long off0, long long stride, int n) {
        __syncthreads();
        const int tot = n * K * (NB + 1);
        for (int e = tid; e < tot; e += bd) {
            const int q = e / (K * (NB + 1)), rem = e - q * K * (NB + 1);
            const int ee = rem / K, kk = rem - ee * K;
            const int cc = tile * K + kk;
            R v = R(0);
            if (cc < C) {
                const double T = Tsrc[off0 - q * stride + cc];
                R x;
                if constexpr (MIXED) x = a.c2_over_lam_f[ee] * rcp(float(T));
                else x = a.c2_over_lam[ee] / T;
                v = planck_edge<R>(x);
            }
            s_pl[(q * K + kk) * (NB + 1) + ee] = v;
        }
        __syncthreads();
    };
    // This lane's bin radiance from row q of the chunk, at temperature T.
    auto lane_B = [&](int q, double Td) -> R {
        const R T = R(Td), T2 = T * T;
        const R *row = s_pl + (q * K + kloc) * (NB + 1);
        R I = planck_combine<R>(row[b], row[b + 1]);
        if constexpr (MIXED) {
            const R iT = rcp(T);
            const R xb = a.c2_over_lam_f[b] * iT, xa = a.c2_over_lam_f[b + 1] * iT;
            if (xb - xa <= R(0.5)) I = planck_gl3<R>(xa, xb);
        }
        return R(kPref) * T2 * T2 * I;
    };

    double mu = 0.0;
    bool day = false;
    if (active) {
        mu = a.mu[c];
        day = mu > 0.0;
        if (!isfinite(mu)) fl |= F_INVALID;
        double ti = a.Tint[c];
        if (!(ti >= 0.0) || !isfinite(ti)) fl |= F_INVALID;
        double T = a.T[(long long)N * C + c];
        if (!(T > 0.0) || !isfinite(T)) fl |= F_INVALID;
    }
    edge_chunk(a.Tint, 0, 0, 1);
    const double Fboa = active ? double(kPI) * double(lane_B(0, a.Tint[c])) : 0.0;

    LaneState st;
    double Fstar_b = 0.0;
    if (active) {
        Fstar_b = a.F_star[b];
        st = lane_top(day, mu, Fstar_b, a.Ftoa ? a.Ftoa[(long long)c * NB + b] : 0.0);
    }
    const double inv_mu = day ? 1.0 / mu : 0.0;
    const double inv_eps2 = 1.0 / a.o.eps2;
    const long long LB = (long long)C * NB;
    const long long L = a.L;
    const long long lane_off = (long long)c * NB + b;

    // inputs of the next layer, loaded one layer ahead of their use
    double nx_dt = 0.0, nx_w = 0.0, nx_g = 0.0, nx_T = 1.0;
    if (active) {
        const long long idx = (long long)(N - 1) * LB + lane_off;
        nx_dt = a.dtau[idx];
        nx_w = a.w0[idx];
        nx_g = a.g0[idx];
        nx_T = a.T[(long long)(N - 1) * C + c];
    }
    R Bup = R(0);
    // levels N, N-1, ..., 0 in chunks of PC; level i closes layer i (between i and i+1)
    for (int s = N; s >= 0; s -= PC) {
        const int n = min(PC, s + 1);
        edge_chunk(a.T, (long long)s * C, C, n);
        for (int q = 0; q < n; ++q) {
            const int i = s - q;
            R B = R(0);
            if (active) B = lane_B(q, a.T[(long long)i * C + c]);
            if (i == N) {
                Bup = B;
                continue;
            }
            if (active) {
                const double dt = nx_dt, w = nx_w, g = nx_g, Tl = nx_T;
                if (i > 0) {
                    const long long idx = (long long)(i - 1) * LB + lane_off;
                    nx_dt = a.dtau[idx];
                    nx_w = a.w0[idx];
                    nx_g = a.g0[idx];
                    nx_T = a.T[(long long)(i - 1) * C + c];
                }
                const BackRec rec = lane_layer<MIXED>(st, dt, w, g, Tl, day, mu, inv_mu, Fstar_b,
                                                      B, Bup, a.o, inv_eps2, fl);
                double *sp = a.scratch + (long long)i * 5 * L + gl;
                sp[0] = rec.G;
                sp[L] = rec.H;
                sp[2 * L] = rec.c;
                sp[3 * L] = rec.d;
                sp[4 * L] = rec.Fb;
            }
            Bup = B;
        }
    }
    __syncthreads();   // the LDS edge rows are reused by the bin sums below

    // BOA condition: F_up_0 - F_dn_0 = F_BOA + F_beam_0, with F_dn_0 = c_0 F_up_0 + d_0
    double Fu = 0.0, Fd = 0.0, Fbi = 0.0;
    if (active) {
        lane_boa(st, Fboa, Fu, Fd, Fbi);
        if (fl) atomicOr(&s_flag[kloc], fl);
    }

    // back-substitution upward, bin sums in chunks of CH interfaces; the
    // record of the next layer is loaded one step ahead of its use
    double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0, r4 = 0.0;
    if (active) {
        const double *sp = a.scratch + gl;
        r0 = sp[0]; r1 = sp[L]; r2 = sp[2 * L]; r3 = sp[3 * L]; r4 = sp[4 * L];
    }
    for (int i0 = 0; i0 <= N; i0 += CH) {
        const int nch = min(CH, N + 1 - i0);
        for (int ii = 0; ii < nch; ++ii) {
            const int i = i0 + ii;
            if (active) {
                if (i > 0) {
                    const double G = r0, H = r1, cj = r2, dj = r3;
                    Fbi = r4;
                    if (i < N) {
                        const double *sp = a.scratch + (long long)i * 5 * L + gl;
                        r0 = sp[0]; r1 = sp[L]; r2 = sp[2 * L]; r3 = sp[3 * L]; r4 = sp[4 * L];
                    }
                    lane_up(G, H, cj, dj, Fu, Fd);
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
            const int cc = tile * K + kk;
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
            const int cc = tile * K + kk;
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
        const int cc = tile * K + kk;
        if (cc < C && a.flags) a.flags[cc] = s_flag[kk];
    }
}

// One request: workgroup = tile.
template <bool MIXED>
__global__ void __launch_bounds__(kMaxThreads) k_solve(const SolveArgs a)
{
    solve_tile<MIXED>(a, blockIdx.x);
}

// Several requests in one launch (serving): workgroup g belongs to the request
// r with first[r] <= g < first[r+1]; all requests share the tile width.
template <bool MIXED>
__global__ void __launch_bounds__(kMaxThreads)
k_solve_batch(const SolveArgs *__restrict__ reqs, const int *__restrict__ first, int n)
{
    const int g = blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {   // last r with first[r] <= g
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    solve_tile<MIXED>(reqs[lo], g - first[lo]);
}

}  // namespace

int default_cols_per_block(int C, int NB)
{
    int K = 256 / NB;
    if (K < 1) K = 1;
    if (K > C) K = C;
    return K;
}

Geometry solve_geometry(int C, int NB, int K)
{
    Geometry g;
    g.K = K > 0 ? K : default_cols_per_block(C, NB);
    if (g.K > C) g.K = C;
    int lanes = g.K * NB;
    g.threads = ((lanes + 63) / 64) * 64;
    g.blocks = (C + g.K - 1) / g.K;
    g.lanes = (long long)g.blocks * g.threads;
    const int ch = chunk_for(g.threads, g.K, NB);
    const size_t front = std::max((size_t)3 * ch * g.threads, (size_t)PC * g.K * (NB + 1));
    g.lds = front * 8 + (size_t)g.K * (ch + 1) * 8 + (size_t)g.K * 4;
    return g;
}

size_t solve_scratch_bytes(int C, int N, int NB, int K)
{
    Geometry g = solve_geometry(C, NB, K);
    return (size_t)N * 5 * (size_t)g.lanes * sizeof(double);
}

hipError_t launch_solve_batch(const SolveArgs *d_reqs, const int *d_first, int n, int total_blocks,
                              int threads, size_t lds, int precision, hipStream_t s)
{
    if (precision == 1)
        hipLaunchKernelGGL(k_solve_batch<true>, dim3(total_blocks), dim3(threads), lds, s, d_reqs,
                           d_first, n);
    else
        hipLaunchKernelGGL(k_solve_batch<false>, dim3(total_blocks), dim3(threads), lds, s, d_reqs,
                           d_first, n);
    return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs &a, int precision, hipStream_t s)
{
    Geometry g = solve_geometry(a.C, a.NB, a.K);
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

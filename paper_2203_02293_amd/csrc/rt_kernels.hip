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
#include "rt_wave.hpp"

#include <math.h>
#include <algorithm>
#include <type_traits>

namespace rtk {
namespace {

// LDS chunk of interfaces reduced at once over bins
__host__ __device__ constexpr int lds_budget() { return 60 * 1024; }

constexpr int PC = 8;   // lane kernel: levels whose Planck edges are computed per barrier

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
template <bool MIXED, bool IN32>
__device__ __forceinline__ void solve_tile_lane(const SolveArgs &a, const int tile)
{
    using R = typename std::conditional<MIXED, float, double>::type;
    // storage type of dtau, w0, g0 (FP32 on the mixed path only); loaded ahead
    // in it and turned into FP64 where used, so no load is waited for early
    using InT = typename std::conditional<IN32, float, double>::type;
    const InT *const in_dt = reinterpret_cast<const InT *>(a.dtau);
    const InT *const in_w = reinterpret_cast<const InT *>(a.w0);
    const InT *const in_g = reinterpret_cast<const InT *>(a.g0);
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
    // per-bin tables in LDS (no global load inside the layer loop; see the
    // layer kernel): c2/lambda at the edges in FP64 and FP32, F*
    double *s_c2 = s_fnet + K * (CH + 1);                      // [NB+1]
    double *s_fs = s_c2 + (NB + 1);                            // [NB]
    float *s_c2f = reinterpret_cast<float *>(s_fs + NB);       // [NB+1]
    uint32_t *s_flag = reinterpret_cast<uint32_t *>(s_c2f + (NB + 2));  // [K]

    for (int kk = tid; kk < K; kk += bd) s_flag[kk] = 0u;
    for (int e = tid; e <= NB; e += bd) {
        s_c2[e] = a.c2_over_lam[e];
        s_c2f[e] = a.c2_over_lam_f[e];
        if (e < NB) s_fs[e] = a.F_star[e];
    }
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
                v = planck_edge<R>(s_c2[ee] / T);
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
            const R xb = s_c2f[b] * iT, xa = s_c2f[b + 1] * iT;
            if (planck_narrow(xa, xb)) {
                const double iTd = rcp(Td);
                I = planck_gl3(s_c2[b + 1] * iTd, s_c2[b] * iTd);
            }
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

    ElimState st = elim_top(0.0);
    double Fstar_b = 0.0;
    if (active) {
        Fstar_b = s_fs[b];
        st = elim_top(a.Ftoa ? a.Ftoa[(long long)c * NB + b] : 0.0);
    }
    const double inv_mu = day ? 1.0 / mu : 0.0;
    const double muF = day ? mu * Fstar_b : 0.0;
    double Fb_up = muF, tau = 0.0;   // beam at the current interface, tau_N = 0
    const double inv_eps2 = 1.0 / a.o.eps2;
    const long long LB = (long long)C * NB;
    const long long L = a.L;
    const long long lane_off = (long long)c * NB + b;

    // inputs of the next layer, loaded one layer ahead of their use
    InT nx_dt = InT(0), nx_w = InT(0), nx_g = InT(0);
    double nx_T = 1.0;
    if (active) {
        const long long idx = (long long)(N - 1) * LB + lane_off;
        nx_dt = in_dt[idx];
        nx_w = in_w[idx];
        nx_g = in_g[idx];
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
                const double dt = double(nx_dt), w = double(nx_w), g = double(nx_g), Tl = nx_T;
                if (i > 0) {
                    const long long idx = (long long)(i - 1) * LB + lane_off;
                    nx_dt = in_dt[idx];
                    nx_w = in_w[idx];
                    nx_g = in_g[idx];
                    nx_T = a.T[(long long)(i - 1) * C + c];
                }
                if (!(Tl > 0.0) || !isfinite(Tl)) fl |= F_INVALID;
                double Fb_lo = 0.0;
                if (day) {
                    tau += dt;   // summed from the TOA, as the optical depth is defined
                    Fb_lo = beam_at<MIXED>(muF, tau, inv_mu);
                }
                const Layer<R> Ly = layer_item<MIXED, R, MIXED>(dt, w, g, day, mu, inv_mu, Fb_up, Fb_lo, B,
                                                         Bup, a.o, inv_eps2, fl);
                const BackRec rec = elim_step(st, double(Ly.t), double(Ly.r), double(Ly.omr),
                                              double(Ly.A), double(Ly.Sup), double(Ly.Sdn));
                double *sp = a.scratch + (long long)i * 5 * L + gl;
                sp[0] = rec.G;
                sp[L] = rec.H;
                sp[2 * L] = rec.c;
                sp[3 * L] = rec.d;
                sp[4 * L] = Fb_up;
                Fb_up = Fb_lo;
            }
            Bup = B;
        }
    }
    __syncthreads();   // the LDS edge rows are reused by the bin sums below

    // BOA condition: F_up_0 - F_dn_0 = F_BOA + F_beam_0, with F_dn_0 = c_0 F_up_0 + d_0
    double Fu = 0.0, Fd = 0.0, Fbi = 0.0;
    if (active) {
        elim_boa(st, Fboa, Fb_up, Fu, Fd);
        Fbi = Fb_up;
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
                    back_step(G, H, cj, dj, Fu, Fd);
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
        if (cc >= C) continue;
        if (a.flags) a.flags[cc] = s_flag[kk];
        const uint32_t bad = status_bits(s_flag[kk]);
        if (a.status && bad) atomicOr(a.status, bad);
    }
}

// ---------------------------------------------------------------------------
// Layer kernel.  A workgroup holds K whole columns (T = K NB lanes) and walks
// the levels from the TOA in chunks of PC.  Each chunk goes through
//   E  Planck edge integrals of its levels (per column and bin edge),
//   V  level items (level, lane): bin radiance from the edge integrals and the
//      direct beam from the optical depth summed down from the TOA,
//   Y  layer items (layer, lane): coefficients and normalised sources,
//   Z  the FP64 elimination through its layers, one sweep thread per lane,
//      which writes the back-substitution records,
// in a software pipeline with one barrier per chunk: phase m runs Z of chunk
// m, Y of m+1, V of m+2 and E of m+3, so the elimination's dependent chain
// overlaps the other threads' transcendental work.  Items of E, V and Y are
// spread over all threads of the workgroup, so that work runs at full
// occupancy even when the grid holds few (column, bin) lanes.  The records
// are 32 bytes per (layer, lane) (G, H, c, d); the back-substitution reads
// them back in passes of CH interfaces, staged in LDS one pass ahead by all
// threads, and closes each pass with its bin sums.
// ---------------------------------------------------------------------------
// Workgroup size bound of the layer kernel: FP64 items need ~170 VGPRs, which
// three wavefronts per SIMD can hold; the FP32 items fit four.
__host__ __device__ constexpr int layer_max_threads(bool mixed) { return mixed ? 1024 : 768; }
// Items per thread and phase (level or layer items of a chunk).  One: a second
// item's prefetch registers push the FP32 kernel past 128 VGPRs and into
// spills, which costs more than the extra barriers of shorter chunks.
__host__ __device__ constexpr int layer_items_per_thread(bool) { return 1; }
// Back-substitution records (2 x 16 bytes per layer and lane) that one thread
// stages per pass: bounds the interfaces per pass, CH, by 2 CH T <= kBackUnits W.
constexpr int kBackUnits = 8;

struct LpLayout {
    size_t flag, mu, wl, tab, part, np;                // persistent
    size_t F, dt, Tl, tau, B, rec, rfl, edge, front;   // forward sweep
    size_t red, brec, back;                            // back-substitution (aliases the forward)
    size_t total;
};

__host__ __device__ inline size_t lp_align(size_t x) { return (x + 15) & ~size_t(15); }

// NB: lanes per column (bins x Gaussian points), NBR: bins (Planck edges NBR+1)
// Whether the back-substitution sums bins within wavefronts: 8..64 lanes per
// column, padded to a power of two NBp, with K NBp <= W.
__host__ __device__ inline int pow2_at_least(int n)
{
    int p = 1;
    while (p < n) p *= 2;
    return p;
}
__host__ __device__ inline bool layer_wsum(int K, int NB, int W)
{
    const int NBp = pow2_at_least(NB);
    return NB >= 8 && NBp <= 64 && K * NBp <= W;
}

__host__ __device__ inline LpLayout lp_layout(int K, int NB, int NBR, int PC, int CH, bool mixed,
                                              bool wsum = false)
{
    const size_t T = (size_t)K * NB, rs = mixed ? 4 : 8;
    LpLayout L;
    size_t o = 0;
    L.flag = o; o += lp_align(4 * (size_t)K);
    L.mu = o;   o += lp_align(8 * 3 * (size_t)K);              // mu, 1/mu, T_int per column
    L.wl = o;   o += lp_align(8 * (size_t)NB);                 // weight of each lane of a column
    // per-bin tables (c2/lambda at the edges in FP64 and FP32, F*): in LDS so
    // that no phase waits on a global load of its own (the input prefetches
    // issued before it would drain with it: the vector-memory counter is in order)
    L.tab = o;  o += lp_align(8 * (size_t)(NBR + 1) + 8 * (size_t)NBR + 4 * (size_t)(NBR + 1));
    // partial sums of the column sums, 2 buffers: a chunk's beam partials
    // (at most W of them) are written while the previous chunk's are summed
    size_t np = 1024;
    if ((size_t)2 * CH * K > np) np = (size_t)2 * CH * K;
    if ((size_t)K > np) np = (size_t)K;                        // (prologue: T at level N per column)
    L.np = np;
    L.part = o; o += lp_align(8 * 2 * np);
    const size_t base = o;
    L.F = o;    o += lp_align(8 * 2 * (PC + 1) * T);      // beam: 2 blocks of levels, row 0 = chunk top
    L.dt = o;   o += lp_align(8 * 2 * (size_t)PC * T);    // dtau of a chunk's layers, 2 buffers
    L.Tl = o;   o += lp_align(8 * 3 * (size_t)PC * K);    // T of a chunk's levels, 3 slots
    L.tau = o;  o += lp_align(8 * 2 * T);                 // optical depth at the chunk top (2 buffers)
    L.B = o;    o += lp_align(rs * 2 * (PC + 1) * T);     // Planck bin radiance, blocks as F
    L.rec = o;  o += lp_align(rs * 2 * 6 * PC * T);       // t r omr A S_up S_dn per layer, 2 buffers
    L.rfl = o;  o += lp_align(4 * 2 * PC * T);            // flags per layer, 2 buffers
    L.edge = o; o += lp_align(rs * (2 * PC + 2) * K * (NBR + 1));   // Planck edge integrals, 2 buffers + T_int, T_N rows
    L.front = o;
    size_t ob = base;
    if (wsum) {   // records in registers: only the level-0 fluxes pass through LDS
        L.red = ob;
        L.brec = ob; ob += lp_align(8 * 2 * T);
    } else {
        L.red = ob;  ob += lp_align(8 * 2 * (size_t)CH * T);  // F_up, F_dn of CH levels
        L.brec = ob; ob += lp_align(16 * 2 * (size_t)CH * T); // records of CH layers
    }
    L.back = ob;
    L.total = L.front > L.back ? L.front : L.back;
    return L;
}

// status: where the tile ORs the condition bits that fail a request (a.status,
// or the serving worker's word for the tile), or NULL.  KARG: ka is the same
// arguments in the constant address space (see args() below); otherwise ka is
// unused.
template <bool MIXED, bool IN32, bool KARG>
__device__ __forceinline__ void solve_tile_layer(const SolveArgs &a, const int tile,
                                                 uint32_t *const status, ArgsK ka)
{
    using R = typename std::conditional<MIXED, float, double>::type;
    // storage type of dtau, w0, g0 (FP32 on the mixed path only); loaded ahead
    // in it and turned into FP64 where used, so no load is waited for early
    using InT = typename std::conditional<IN32, float, double>::type;
    // The fields read inside the loops come through args(): with KARG from ka
    // (ArgsK), made opaque (fresh()) at the top of each pass of a loop; without
    // KARG (the serving worker, whose copy of the arguments is written inside
    // the kernel and so is not read through the scalar cache) from a.
    ArgsK ap = ka;
    auto fresh = [&]() {
        if constexpr (KARG) opaque_args(ap);
    };
    auto args = [&]() -> const SolveArgs & {
        if constexpr (KARG) return *(const SolveArgs *)ap;
        else return a;
    };
    // the layer inputs: without KARG their pointers are taken once, here (a
    // read of a's fields after the kernel's own stores is a load again)
    const InT *const in_dt0 = reinterpret_cast<const InT *>(a.dtau);
    const InT *const in_w0 = reinterpret_cast<const InT *>(a.w0);
    const InT *const in_g0 = reinterpret_cast<const InT *>(a.g0);
    auto in_dt = [&]() -> const InT * {
        if constexpr (KARG) return reinterpret_cast<const InT *>(args().dtau);
        else return in_dt0;
    };
    auto in_w = [&]() -> const InT * {
        if constexpr (KARG) return reinterpret_cast<const InT *>(args().w0);
        else return in_w0;
    };
    auto in_g = [&]() -> const InT * {
        if constexpr (KARG) return reinterpret_cast<const InT *>(args().g0);
        else return in_g0;
    };
    extern __shared__ double smem[];
    char *lds = reinterpret_cast<char *>(smem);
    const int NB = a.NB, K = a.K, C = a.C, N = a.N, PC = a.PC, CH = a.CH;
    const int NG = a.NG, NBR = NB / NG;   // lanes per column = bins x Gaussian points
    const int T = K * NB;
    const int tid = threadIdx.x, W = blockDim.x;
    const bool wsum = layer_wsum(K, NB, W);
    const LpLayout Lo = lp_layout(K, NB, NBR, PC, CH, MIXED, wsum);
    uint32_t *s_flag = reinterpret_cast<uint32_t *>(lds + Lo.flag);   // [K]
    double *s_mu = reinterpret_cast<double *>(lds + Lo.mu);           // [3][K]: mu, 1/mu, T_int
    double *s_wl = reinterpret_cast<double *>(lds + Lo.wl);           // [NB]
    double *s_c2 = reinterpret_cast<double *>(lds + Lo.tab);          // [NBR+1] c2 / lambda edge
    double *s_fs = s_c2 + (NBR + 1);                                  // [NBR] F* per bin
    float *s_c2f = reinterpret_cast<float *>(s_fs + NBR);             // [NBR+1] FP32 c2 / lambda
    double *s_part = reinterpret_cast<double *>(lds + Lo.part);       // [2][np] partial column sums
    double *s_F0 = reinterpret_cast<double *>(lds + Lo.F);            // [2][PC+1][T]
    double *s_dt0 = reinterpret_cast<double *>(lds + Lo.dt);          // [2][PC][T]
    double *s_T0 = reinterpret_cast<double *>(lds + Lo.Tl);           // [3][PC][K]
    double *s_tau = reinterpret_cast<double *>(lds + Lo.tau);         // [2][T]
    R *s_B0 = reinterpret_cast<R *>(lds + Lo.B);                      // [2][PC+1][T]
    R *s_rec0 = reinterpret_cast<R *>(lds + Lo.rec);                  // [2][6][PC][T]
    uint32_t *s_rfl0 = reinterpret_cast<uint32_t *>(lds + Lo.rfl);    // [2][PC][T]
    R *s_edge0 = reinterpret_cast<R *>(lds + Lo.edge);                // [2 PC + 2][K][NBR+1]
    double *s_red = reinterpret_cast<double *>(lds + Lo.red);         // [2][CH][T]

    const int c0 = tile * K;                    // first column of the tile
    const long long LB = (long long)C * NB;     // one layer of a [C][NB] plane
    const long long toff = (long long)c0 * NB;  // lane 0 of the tile in such a plane
    const long long L = a.L;
    const double inv_eps2 = 1.0 / a.o.eps2;

    // the sweep lane of this thread
    const bool sweep = tid < T;
    const int kl = sweep ? tid / NB : 0, bl = tid - kl * NB;
    const bool active = sweep && (c0 + kl < C);
    const long long gl = (long long)tile * T + tid;
    uint32_t fl = 0u;

    // this thread's items of the level and layer phases (the launch has
    // PC T <= IT W): item k is tid + k W, row iq of the chunk, lane il =
    // (column ikk, lane ib of the column, bin irb); and its level-temperature
    // slots (row tq, column tkk)
    constexpr int IT = layer_items_per_thread(MIXED);
    int iq[IT], il[IT], ikk[IT], irb[IT], tq[IT], tkk[IT];
    bool icol[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const int e = tid + k * W;
        iq[k] = e / T;
        il[k] = e - iq[k] * T;
        ikk[k] = il[k] / NB;
        const int ib = il[k] - ikk[k] * NB;
        irb[k] = NG == 1 ? ib : ib / NG;
        icol[k] = c0 + ikk[k] < C;
        tq[k] = e / K;
        tkk[k] = e - tq[k] * K;
    }
    // Item offset of this thread within a round of W items (edge integrals,
    // beam totals): the sweep threads (tid < T) take the last T offsets, so a
    // partial round leaves them, busy with the elimination, out.
    const int rot = (tid + W - T) % W;
    // this thread's edge items (offsets rot + k W of a chunk's edges; a chunk has
    // at most 2 IT W of them: K (NBR + 1) <= 2 T per level)
    const int per = K * (NBR + 1);
    int eq[2 * IT], eee[2 * IT], ekk[2 * IT];
#pragma unroll
    for (int k = 0; k < 2 * IT; ++k) {
        const int e = rot + k * W, q = e / per, rem = e - q * per;
        eq[k] = q;
        eee[k] = rem / K;
        ekk[k] = rem - eee[k] * K;
    }


    // Temperature of level l and the bin-summed output slot of level l: on the
    // sub-layer grid even levels are interfaces and odd levels layer centres.
    const bool sub = a.sub != 0;
    // both temperature pointers read as uniform values, then one chosen per
    // lane (a per-lane choice between the two argument fields would load the
    // chosen pointer with a vector load and wait for it, and with it for every
    // prefetch in flight)
    const double *const T_if0 = a.T, *const T_ce0 = sub ? a.Tc : a.T;
    auto T_at = [&](int l, int cc) -> double {
        const double *T_if = T_if0, *T_ce = T_ce0;
        if constexpr (KARG) {
            T_if = args().T;
            T_ce = sub ? args().Tc : args().T;
        }
        const double *base = (sub && (l & 1)) ? T_ce : T_if;
        return base[(long long)(sub ? (l >> 1) : l) * C + cc];
    };
    auto out_at = [&](double *iface, double *centre, int l, int cc) -> double * {
        if (sub) return ((l & 1) ? centre : iface) + (long long)(l >> 1) * C + cc;
        return iface + (long long)l * C + cc;
    };

    // Planck edge integrals of n levels into rows 0..n-1 of edge buffer s_edge,
    // edge-major so a wavefront's lanes share one edge; temperatures from
    // Ts[q][K] (LDS).
    auto edges = [&](R *s_edge, const double *Ts, int n) {
#pragma unroll
        for (int k = 0; k < 2 * IT; ++k) {
            if (eq[k] >= n) continue;
            const int q = eq[k], ee = eee[k], kk = ekk[k];
            const int cc = c0 + kk;
            R v = R(0);
            if (cc < C) {
                v = planck_edge<R>(s_c2[ee] * rcp(Ts[q * K + kk]));
            }
            s_edge[(q * K + kk) * (NBR + 1) + ee] = v;
        }
    };
    // Bin radiance of (column kk, bin b) from row q of edge buffer s_edge at
    // temperature Td.
    auto bin_B = [&](const R *s_edge, int q, int kk, int b, double Td) -> R {
        const R Tr = R(Td), T2 = Tr * Tr;
        const R *row = s_edge + (q * K + kk) * (NBR + 1);
        R I = planck_combine<R>(row[b], row[b + 1]);
        if constexpr (MIXED) {
            const R iT = rcp(Tr);
            const R xb = s_c2f[b] * iT, xa = s_c2f[b + 1] * iT;
            if (planck_narrow(xa, xb)) {
                const double iTd = rcp(Td);
                I = planck_gl3(s_c2[b + 1] * iTd, s_c2[b] * iTd);
            }
        }
        return R(kPref) * T2 * T2 * I;
    };
    // Column sums of nrows rows of lanes (row r of column kk at src + r rstride +
    // kk NB), weighted by the Gaussian points' weights, in two steps with a
    // barrier between: (1) P partial sums per (row, column), partial p over the
    // lanes p, p+P, ... in order; (2) the P partials in order.  Fixed order, so
    // repeated solves are bitwise identical.
    // P balances the two serial steps (about sqrt(NB) each) within the threads.
    int Psq = 1;
    while ((Psq + 1) * (Psq + 1) <= NB) ++Psq;
    auto colsum_P = [&](int nrows) -> int {
        const int cap = W / (nrows * K);
        return Psq > cap ? (cap < 1 ? 1 : cap) : Psq;
    };
    auto colsum_partials = [&](double *part, const double *src, int rstride, int nrows, int P) {
        for (int t = tid; t < nrows * K * P; t += W) {
            const int r = t / (K * P), rem = t - r * (K * P);
            const int kk = rem / P, p = rem - kk * P;
            const double *row = src + (size_t)r * rstride + kk * NB;
            double sum = 0.0;
            if (NG == 1) {
                for (int b = p; b < NB; b += P) sum += row[b];
            } else {
                for (int b = p; b < NB; b += P) sum += s_wl[b] * row[b];
            }
            part[t] = sum;
        }
    };
    auto colsum_total = [&](const double *part, int r, int kk, int P) -> double {
        const double *pp = part + ((size_t)r * K + kk) * P;
        double sum = 0.0;
        for (int p = 0; p < P; ++p) sum += pp[p];
        return sum;
    };

    // Chunks of levels from the TOA: chunk m has top level s_m = N - m PC and
    // n_m = min(PC, s_m) levels s_m - 1 .. s_m - n_m below it (and the layers
    // between); NCH chunks in all.  Each chunk passes through
    //   E(m)  Planck edge integrals of its levels,
    //   V(m)  level items: bin radiance and direct beam of its levels (rows
    //         1..n of its row block; row 0 is the last level of chunk m-1),
    //   Y(m)  layer items: coefficients and normalised sources of its layers,
    //   Z(m)  the FP64 elimination through its layers (sweep threads),
    // and its beam bin sums (partials, then totals).  Phase m of the loop runs
    // Z(m), Y(m+1), V(m+2) and E(m+3), the partials of chunk m+1 and the
    // totals of chunk m, with one barrier at its end.  Buffers, by chunk
    // parity unless noted: row blocks s_B/s_F, edge rows, layer records,
    // dtau rows, beam partials; level temperatures in slot m % 3.  dtau, w0
    // and g0 of an item are loaded by the thread that owns the item; w0 and
    // g0 stay in its registers, dtau goes to LDS for the optical-depth sums.
    const int NCH = (N + PC - 1) / PC;
    auto ctop = [&](int m) { return N - m * PC; };
    auto cn = [&](int m) { return m < NCH ? min(PC, N - m * PC) : 0; };
    auto blockB = [&](int m) { return s_B0 + (size_t)(m & 1) * (PC + 1) * T; };
    auto blockF = [&](int m) { return s_F0 + (size_t)(m & 1) * (PC + 1) * T; };
    auto ebuf = [&](int m) { return s_edge0 + (size_t)(m & 1) * PC * K * (NBR + 1); };
    auto tslot = [&](int m) { return s_T0 + (size_t)(m % 3) * PC * K; };
    auto dbuf = [&](int m) { return s_dt0 + (size_t)(m & 1) * PC * T; };
    auto rbuf = [&](int m) { return s_rec0 + (size_t)(m & 1) * 6 * PC * T; };
    auto fbuf = [&](int m) { return s_rfl0 + (size_t)(m & 1) * PC * T; };
    auto pbuf = [&](int m) { return s_part + (size_t)(m & 1) * Lo.np; };

    // this thread's item of chunk m: input index, and its level-temperature slot
    auto item_idx = [&](int m) -> long long {
        return (long long)(ctop(m) - 1 - iq[0]) * LB + toff + il[0];
    };
    auto has_item = [&](int m) { return iq[0] < cn(m) && icol[0]; };
    auto load_dt = [&](int m) -> InT {
        return has_item(m) ? in_dt()[item_idx(m)] : InT(0);
    };
    auto load_wg = [&](int m, InT &w, InT &g) {
        w = g = InT(0);
        if (has_item(m)) {
            const long long idx = item_idx(m);
            w = in_w()[idx];
            g = in_g()[idx];
        }
    };
    auto load_T = [&](int m) -> double {
        return (tq[0] < cn(m) && c0 + tkk[0] < C) ? T_at(ctop(m) - 1 - tq[0], c0 + tkk[0]) : 1.0;
    };
    auto store_dt = [&](int m, InT v) {
        if (iq[0] < cn(m)) dbuf(m)[iq[0] * T + il[0]] = double(v);
    };
    auto store_T = [&](int m, double v) { if (tq[0] < cn(m)) tslot(m)[tid] = v; };

    // V(m): the carry of chunk m-1's last level into row 0, then this thread's
    // level item (rows 1..n), and the optical depth at the top of chunk m+1
    auto level_items = [&](int m) {
        const int n = cn(m);
        if (m > 0 && tid < T) {
            blockB(m)[tid] = blockB(m - 1)[(size_t)cn(m - 1) * T + tid];
            blockF(m)[tid] = blockF(m - 1)[(size_t)cn(m - 1) * T + tid];
        }
        if (iq[0] >= n) return;
        const int q = iq[0], l = il[0], kk = ikk[0], rb = irb[0];
        const double *dt = dbuf(m);
        R B = R(0);
        double Fb = 0.0;
        if (icol[0]) {
            const double Tv = tslot(m)[q * K + kk];
            if (!(Tv > 0.0) || !isfinite(Tv)) atomicOr(&s_flag[kk], (uint32_t)F_INVALID);
            B = bin_B(ebuf(m), q, kk, rb, Tv);
            const double mu = s_mu[kk];
            if (mu > 0.0) {
                double tau = s_tau[(m & 1) * T + l];
                // from the TOA down; the row pointer steps through the rows (a
                // hoisted address per row would be spilled, and a spill reload
                // waits for every global load in flight)
                const double *dp = dt + l;
#pragma unroll 1
                for (int qq = 0; qq <= q; ++qq, dp += T) tau += *dp;
                Fb = beam_at<MIXED>(mu * s_fs[rb], tau, s_mu[K + kk]);
                if (q == n - 1) s_tau[((m + 1) & 1) * T + l] = tau;
            }
        }
        blockB(m)[(q + 1) * T + l] = B;
        blockF(m)[(q + 1) * T + l] = Fb;
    };
    // Y(m): this thread's layer item, w0 and g0 from its registers
    auto layer_items = [&](int m, InT wr, InT gr) {
        const double w = double(wr), g = double(gr);
        const int n = cn(m);
        if (iq[0] >= n) return;
        const int q = iq[0], l = il[0], kk = ikk[0];
        const R *cB = blockB(m);
        const double *cF = blockF(m);
        uint32_t f = 0u;
        Layer<R> Ly{};
        if (icol[0]) {
            const double mu = s_mu[kk];
            Ly = layer_item<MIXED, R, MIXED>(dbuf(m)[q * T + l], w, g, mu > 0.0, mu, s_mu[K + kk],
                                      cF[q * T + l], cF[(q + 1) * T + l], cB[(q + 1) * T + l],
                                      cB[q * T + l], args().o, inv_eps2, f);
        }
        R *rp = rbuf(m) + (size_t)q * T + l;
        const size_t ps = (size_t)PC * T;
        rp[0] = Ly.t;
        rp[ps] = Ly.r;
        rp[2 * ps] = Ly.omr;
        rp[3 * ps] = Ly.A;
        rp[4 * ps] = Ly.Sup;
        rp[5 * ps] = Ly.Sdn;
        fbuf(m)[q * T + l] = f;
    };
    // beam bin sums of chunk m's levels: rows 1..n (rows 0..n in chunk 0,
    // whose row 0 is level N)
    auto beam_rows = [&](int m, int &r0, int &nr) {
        r0 = m == 0 ? 0 : 1;
        nr = cn(m) + 1 - r0;
    };
    auto beam_partials = [&](int m) {
        int r0, nr;
        beam_rows(m, r0, nr);
        colsum_partials(pbuf(m), blockF(m) + (size_t)r0 * T, T, nr, colsum_P(nr));
    };
    auto beam_totals = [&](int m) {
        int r0, nr;
        beam_rows(m, r0, nr);
        const int P = colsum_P(nr);
        for (int t = rot; t < nr * K; t += W) {
            const int q = t / K, kk = t - q * K;
            if (c0 + kk < C)
                *out_at(args().F_beam, args().F_beam_c, ctop(m) - r0 - q, c0 + kk) = colsum_total(pbuf(m), q, kk, P);
        }
    };

    // Prologue.  Its global inputs are loaded at once: per column mu, T_int
    // and T at level N, the level temperatures of chunks 0..3, dtau of chunks
    // 0..2, w0 and g0 of chunks 0 and 1, and the TOA downward flux of the
    // sweep lanes.  Then E(0), E(1); V(0); V(1), Y(0), E(2) and chunk 0's beam
    // partials, each step behind a barrier.
    double *s_TN = s_part;       // [K] T at level N (the partial sums are not in use
                                 // before the last prologue step)
    double *s_Ti = s_mu + 2 * K; // [K] T_int
    R *ebuf_x = s_edge0 + (size_t)2 * PC * K * (NBR + 1);   // T_int edge row
    R *ebuf_n = ebuf_x + (size_t)K * (NBR + 1);             // level N edge row
    const double ftoa = (active && a.Ftoa) ? a.Ftoa[toff + tid] : 0.0;
    InT w_c, g_c, w_n, g_n;      // w0, g0 of this thread's items of the next two Y phases
    InT dt_p;                    // dtau loaded ahead, stored later
    double T_p;                  // level temperature loaded ahead, stored later
    {
        const InT d0 = load_dt(0), d1 = load_dt(1);
        const double t0 = load_T(0), t1 = load_T(1), t2 = load_T(2);
        load_wg(0, w_c, g_c);
        load_wg(1, w_n, g_n);
        dt_p = load_dt(2);
        T_p = load_T(3);
        for (int kk = tid; kk < K; kk += W) {
            const int cc = c0 + kk;
            double mu = 0.0, ti = 1.0, tn = 1.0;
            uint32_t f0 = 0u;
            if (cc < C) {
                mu = a.mu[cc];
                ti = a.Tint[cc];
                tn = T_at(N, cc);
                if (!isfinite(mu)) f0 |= F_INVALID;
                if (!(ti >= 0.0) || !isfinite(ti)) f0 |= F_INVALID;
            }
            s_mu[kk] = mu;
            s_mu[K + kk] = mu > 0.0 ? 1.0 / mu : 0.0;
            s_flag[kk] = f0;
            s_TN[kk] = tn;
            s_Ti[kk] = ti;
        }
        for (int b = tid; b < NB; b += W) s_wl[b] = NG == 1 ? 1.0 : a.wg[b % NG];
        for (int e = tid; e <= NBR; e += W) {
            s_c2[e] = a.c2_over_lam[e];
            s_c2f[e] = a.c2_over_lam_f[e];
            if (e < NBR) s_fs[e] = a.F_star[e];
        }
        if (tid < T) s_tau[tid] = 0.0;
        store_dt(0, d0);
        store_dt(1, d1);
        store_T(0, t0);
        store_T(1, t1);
        store_T(2, t2);
    }
    __syncthreads();
    // edge integrals of T_int, level N, and chunks 0 and 1, spread evenly over
    // the threads: row 0 T_int, row 1 level N, then the chunks' level rows
    {
        const int n0 = cn(0), nrow = 2 + n0 + cn(1);
        for (int e = rot; e < nrow * per; e += W) {
            const int r = e / per, rem = e - r * per, ee = rem / K, kk = rem - ee * K;
            const double *Ts;
            R *dst;
            if (r == 0) {
                Ts = s_Ti;
                dst = ebuf_x;
            } else if (r == 1) {
                Ts = s_TN;
                dst = ebuf_n;
            } else {
                const int m = r - 2 < n0 ? 0 : 1, q = r - 2 - (m ? n0 : 0);
                Ts = tslot(m) + q * K;
                dst = ebuf(m) + (size_t)q * K * (NBR + 1);
            }
            R v = R(0);
            if (c0 + kk < C) {
                v = planck_edge<R>(s_c2[ee] * rcp(Ts[kk]));
            }
            dst[kk * (NBR + 1) + ee] = v;
        }
    }
    __syncthreads();
    // level N (row 0 of block 0: item iq = 0, il = tid) and V(0)
    if (tid < T) {
        R B = R(0);
        double Fb = 0.0;
        if (icol[0]) {
            const double Tv = s_TN[ikk[0]];
            if (!(Tv > 0.0) || !isfinite(Tv)) atomicOr(&s_flag[ikk[0]], (uint32_t)F_INVALID);
            B = bin_B(ebuf_n, 0, ikk[0], irb[0], Tv);
            const double mu = s_mu[ikk[0]];
            if (mu > 0.0) Fb = mu * s_fs[irb[0]];
        }
        blockB(0)[tid] = B;
        blockF(0)[tid] = Fb;
    }
    level_items(0);
    __syncthreads();
    if (NCH > 1) level_items(1);
    layer_items(0, w_c, g_c);
    if (NCH > 2) edges(ebuf(2), tslot(2), cn(2));
    beam_partials(0);
    store_dt(2, dt_p);   // (after this thread's Y(0) read of its chunk 0 dtau)
    store_T(3, T_p);
    w_c = w_n;
    g_c = g_n;
    dt_p = load_dt(3);
    T_p = load_T(4);
    __syncthreads();

    ElimState st = elim_top(ftoa);
    for (int m = 0; m < NCH; ++m) {
        const int s = ctop(m), n = cn(m);
        fresh();
        // Z(m)
        if (active) {
            const R *rb0 = rbuf(m);
            const uint32_t *fb0 = fbuf(m);
            const size_t ps = (size_t)PC * T;
            // the LDS record of layer q + 1 is read while layer q is eliminated
            // (the last read repeats layer n - 1 and is unused)
            const R *rp0 = rb0 + tid;
            R x0 = rp0[0], x1 = rp0[ps], x2 = rp0[2 * ps], x3 = rp0[3 * ps], x4 = rp0[4 * ps],
              x5 = rp0[5 * ps];
            uint32_t xf = fb0[tid];
            for (int q = 0; q < n; ++q) {
                const int qn = min(q + 1, n - 1);
                const R *rp = rb0 + (size_t)qn * T + tid;
                const R y0 = rp[0], y1 = rp[ps], y2 = rp[2 * ps], y3 = rp[3 * ps], y4 = rp[4 * ps],
                        y5 = rp[5 * ps];
                const uint32_t yf = fb0[qn * T + tid];
                fl |= xf;
                const BackRec rec = elim_step(st, double(x0), double(x1), double(x2), double(x3),
                                              double(x4), double(x5));
                x0 = y0;
                x1 = y1;
                x2 = y2;
                x3 = y3;
                x4 = y4;
                x5 = y5;
                xf = yf;
                double2 *sp = reinterpret_cast<double2 *>(args().scratch) + ((long long)(s - 1 - q) * L + gl) * 2;
                sp[0] = make_double2(rec.G, rec.H);
                sp[1] = make_double2(rec.c, rec.d);
            }
        }
        beam_totals(m);
        if (m + 1 < NCH) beam_partials(m + 1);
        if (m + 3 < NCH) edges(ebuf(m + 3), tslot(m + 3), cn(m + 3));
        if (m + 2 < NCH) level_items(m + 2);
        // the layer items last, so that their w0, g0 (loaded at the end of the
        // previous phase) have the rest of this phase to arrive
        if (m + 1 < NCH) layer_items(m + 1, w_c, g_c);
        store_dt(m + 3, dt_p);   // (after this thread's Y(m+1) read of its dtau)
        store_T(m + 4, T_p);
        // loads for later phases, into the registers just freed (no copies
        // between registers, which would wait for the loads): w0, g0 of
        // Y(m+2), dtau of V(m+4), T of E(m+5); each has the next phase to land
        load_wg(m + 2, w_c, g_c);
        dt_p = load_dt(m + 4);
        T_p = load_T(m + 5);
        __syncthreads();
    }

    // BOA condition: F_up_0 - F_dn_0 = F_BOA + F_beam_0 (level 0: the last row
    // of the last chunk's block)
    double Fu = 0.0, Fd = 0.0;
    if (active) {
        // F_BOA = pi B_b(T_int) (the T_int edge row stays in LDS)
        const double Fboa = double(kPI) * double(bin_B(ebuf_x, 0, kl, NG == 1 ? bl : bl / NG, s_Ti[kl]));
        elim_boa(st, Fboa, blockF(NCH - 1)[(size_t)cn(NCH - 1) * T + tid], Fu, Fd);
        if (fl) atomicOr(&s_flag[kl], fl);
    }
    __syncthreads();   // the bin-sum buffers alias the forward buffers

    if (wsum) {
        // Back-substitution on a padded layout: thread kk NBp + b takes lane
        // (kk, b), NBp the power of two >= NB, so a column's lanes share a
        // wavefront and the bin sums of each level are wavefront sums
        // (seg_sum2) with no barrier.  Each lane keeps the records of its next RD
        // layers in registers (slot k: the layer below interface i0 + k),
        // loaded RD steps ahead of their use; the loads are unconditional (layer
        // index clamped, a valid lane for the padding) so no slot waits for
        // its load before it is used.  The level-0 fluxes move to the padded
        // layout through LDS; F_net follows in the pass after.
        const int NBp = pow2_at_least(NB);
        const int yk = tid / NBp, yb = tid - yk * NBp, yl = yk * NB + yb;
        const bool yslot = yk < K, yact = yslot && yb < NB && c0 + yk < C;
        double *s_x = reinterpret_cast<double *>(lds + Lo.brec);   // [2][T]
        if (sweep) {
            s_x[tid] = Fu;
            s_x[T + tid] = Fd;
        }
        __syncthreads();
        Fu = yact ? s_x[yl] : 0.0;
        Fd = yact ? s_x[T + yl] : 0.0;
        const double wgt = yact ? s_wl[yb] : 0.0;   // bin-sum weight (0 on padding lanes)
        // the lane of a column segment that holds its sums (seg_sum2) and writes them
        const int ol = NBp <= 16 ? 0 : (NBp == 32 ? 16 : 48);
        const bool outc = yslot && yb == ol && c0 + yk < C;
        // only the wavefronts that hold back-substitution lanes run the steps
        if (wave_uniform(tid >> 6) * 64 < K * NBp) {
            const double2 *rp = reinterpret_cast<const double2 *>(a.scratch) +
                                ((long long)tile * T + (yact ? yl : 0)) * 2;
            // records in flight per lane: 8 in FP64; 4 in the mixed kernel, whose
            // 128 VGPRs then hold the fixed-width sums of 32-lane groups below
            constexpr int RD = MIXED ? 4 : 8;
            double rG[RD], rH[RD], rc[RD], rd[RD];
            auto ld = [&](int j, int k) {
                const double2 *q = rp + (long long)min(j, N - 1) * 2 * L;
                const double2 x = q[0], y = q[1];
                rG[k] = x.x;
                rH[k] = x.y;
                rc[k] = y.x;
                rd[k] = y.y;
            };
#pragma unroll
            for (int k = 1; k < RD; ++k) ld(k - 1, k);
            rG[0] = rH[0] = rc[0] = rd[0] = 0.0;
            // The steps of every level.  NBW: the group width NBp of the bin
            // sums as a compile-time constant (no branches between the DPP
            // steps, so the sums of F_up and F_dn interleave), or 0 for the
            // run-time width.  The mixed kernel fixes only the width 32 (the
            // 30-bin grids): four fixed-width copies of the loop overflow its
            // 128 VGPRs.
            auto levels = [&](auto NBW) {
                constexpr int NW = decltype(NBW)::value;
                for (int i0 = 0; i0 <= N; i0 += RD) {
                    fresh();
#pragma unroll
                    for (int k = 0; k < RD; ++k) {
                        const int i = i0 + k;
                        if (i > N) break;
                        if (yact && i > 0) back_step(rG[k], rH[k], rc[k], rd[k], Fu, Fd);
                        ld(i + RD - 1, k);   // the layer below interface i + RD
                        if (yact) {
                            const long long o = (long long)i * LB + toff + yl;
                            if (args().F_up_bin) args().F_up_bin[o] = Fu;
                            if (args().F_dn_bin) args().F_dn_bin[o] = Fd;
                            if (i == N && args().F_up_toa_bin) {
                                if (NG == 1) args().F_up_toa_bin[toff + yl] = Fu;
                                else s_part[yl] = Fu;   // TOA spectrum, below
                            }
                        }
                        double su = wgt * Fu, sd = wgt * Fd;
                        if constexpr (NW == 0) seg_sum2(su, sd, NBp);
                        else seg_sum2<NW>(su, sd);
                        if (outc) {
                            *out_at(args().F_up, args().F_up_c, i, c0 + yk) = su;
                            *out_at(args().F_dn, args().F_dn_c, i, c0 + yk) = sd;
                        }
                    }
                }
            };
            if (MIXED) {
                if (NBp == 32) levels(std::integral_constant<int, 32>{});
                else levels(std::integral_constant<int, 0>{});
            } else {
                switch (NBp) {   // 8..64 (layer_wsum)
                case 8: levels(std::integral_constant<int, 8>{}); break;
                case 16: levels(std::integral_constant<int, 16>{}); break;
                case 32: levels(std::integral_constant<int, 32>{}); break;
                default: levels(std::integral_constant<int, 64>{}); break;
                }
            }
        }
        __syncthreads();
        // TOA spectrum per bin: the weighted sum over the bin's Gaussian points
        if (NG > 1 && a.F_up_toa_bin) {
            for (int task = tid; task < K * NBR; task += W) {
                const int kk = task / NBR, rb_ = task - kk * NBR, cc = c0 + kk;
                if (cc >= C) continue;
                const double *ru_ = s_part + kk * NB + rb_ * NG;
                double sum = 0.0;
                for (int g = 0; g < NG; ++g) sum += a.wg[g] * ru_[g];
                a.F_up_toa_bin[(long long)cc * NBR + rb_] = sum;
            }
        }
        // net flux of every level (F_up, F_dn and F_beam written above)
        for (int task = tid; task < (N + 1) * K; task += W) {
            const int lev = task / K, kk = task - lev * K, cc = c0 + kk;
            if (cc >= C) continue;
            const double fn = *out_at(a.F_up, a.F_up_c, lev, cc) - *out_at(a.F_dn, a.F_dn_c, lev, cc) -
                              *out_at(a.F_beam, a.F_beam_c, lev, cc);
            *out_at(a.F_net, a.F_net_c, lev, cc) = fn;
            if (!isfinite(fn)) atomicOr(&s_flag[kk], (uint32_t)F_NONFIN);
        }
    } else {
    // back-substitution upward in passes of CH interfaces, each closed by its
    // bin sums.  A pass's records are staged in LDS (s_brec[ii][lane] = (G, H),
    // (c, d) of the layer below interface i0 + ii): every thread loads its
    // share of the next pass's records into registers while the sweep lanes
    // run this pass, and stores them once this pass's records are used.  The
    // loads are unconditional (index clamped to a valid record) so that none
    // of them has to complete before the store.
    constexpr int MU = kBackUnits;
    double2 *s_brec = reinterpret_cast<double2 *>(lds + Lo.brec);   // [CH][T][2]
    const double2 *rec2 = reinterpret_cast<const double2 *>(a.scratch);
    const int units = 2 * CH * T;
    int uii[MU], uoff[MU];   // level in the pass, offset (lane, half) of the unit
#pragma unroll
    for (int k = 0; k < MU; ++k) {
        const int e = min(tid + k * W, units - 1);
        uii[k] = e / (2 * T);
        uoff[k] = (tile * T) * 2 + (e - uii[k] * 2 * T);
    }
    double rx[MU], ry[MU];   // staged units (scalars, so that they stay in registers)
    auto rec_fetch = [&](int i0n) {
#pragma unroll
        for (int k = 0; k < MU; ++k) {
            int jl = i0n + uii[k] - 1;
            if (jl < 0 || jl >= N) jl = 0;
            const double2 v = rec2[(long long)jl * 2 * L + uoff[k]];
            rx[k] = v.x;
            ry[k] = v.y;
        }
    };
    auto rec_store = [&](double2 *dst) {
#pragma unroll
        for (int k = 0; k < MU; ++k)
            if (tid + k * W < units) dst[tid + k * W] = make_double2(rx[k], ry[k]);
    };
    rec_fetch(0);
    rec_store(s_brec);
    __syncthreads();
    const int P = colsum_P(2 * CH);
    for (int i0 = 0; i0 <= N; i0 += CH) {
        fresh();
        const int nch = min(CH, N + 1 - i0);
        rec_fetch(i0 + CH);   // the next pass (clamped, unused, after the last)
        // the beam flux of this thread's first bin-sum task, read ahead
        double fbp = 0.0;
        if (tid < K * nch) {
            const int ii = tid / K, kk = tid - ii * K;
            if (c0 + kk < C) fbp = *out_at(args().F_beam, args().F_beam_c, i0 + ii, c0 + kk);
        }
        for (int ii = 0; ii < nch; ++ii) {
            const int i = i0 + ii;
            if (active) {
                if (i > 0) {
                    const double2 gh = s_brec[(ii * T + tid) * 2], cd = s_brec[(ii * T + tid) * 2 + 1];
                    back_step(gh.x, gh.y, cd.x, cd.y, Fu, Fd);
                }
                const long long o = (long long)i * LB + toff + tid;
                if (args().F_up_bin) args().F_up_bin[o] = Fu;
                if (args().F_dn_bin) args().F_dn_bin[o] = Fd;
                if (i == N && args().F_up_toa_bin && NG == 1) args().F_up_toa_bin[toff + tid] = Fu;
            }
            if (sweep) {
                s_red[(0 * CH + ii) * T + tid] = Fu;
                s_red[(1 * CH + ii) * T + tid] = Fd;
            }
        }
        __syncthreads();
        // outputs of level i0 + ii from its bin sums and the beam sum written
        // by the forward sweep
        auto level_out = [&](int ii, int kk, double su, double sd, double fb) {
            const int lev = i0 + ii, cc = c0 + kk;
            const double fn = su - sd - fb;
            *out_at(args().F_up, args().F_up_c, lev, cc) = su;
            *out_at(args().F_dn, args().F_dn_c, lev, cc) = sd;
            *out_at(args().F_net, args().F_net_c, lev, cc) = fn;
            if (!isfinite(fn)) atomicOr(&s_flag[kk], (uint32_t)F_NONFIN);
        };
        // rows 0..nch-1 hold F_up, rows CH..CH+nch-1 F_dn: both as one block of
        // 2 CH rows (the unused rows of a short pass are summed and ignored)
        colsum_partials(s_part, s_red, T, 2 * CH, P);
        // TOA spectrum per bin: the weighted sum over the bin's Gaussian points
        if (NG > 1 && a.F_up_toa_bin && i0 + nch == N + 1) {
            for (int task = tid; task < K * NBR; task += W) {
                const int kk = task / NBR, rb = task - kk * NBR, cc = c0 + kk;
                if (cc >= C) continue;
                const double *ru_ = s_red + (0 * CH + (N - i0)) * T + kk * NB + rb * NG;
                double sum = 0.0;
                for (int g = 0; g < NG; ++g) sum += a.wg[g] * ru_[g];
                a.F_up_toa_bin[(long long)cc * NBR + rb] = sum;
            }
        }
        if (i0 + CH <= N) rec_store(s_brec);   // this pass's records are used
        __syncthreads();
        // (the next pass writes s_red, read above, and s_part only after its
        // first barrier, so no barrier closes the pass)
        for (int task = tid; task < K * nch; task += W) {
            const int ii = task / K, kk = task - ii * K;
            if (c0 + kk >= C) continue;
            level_out(ii, kk, colsum_total(s_part, ii, kk, P), colsum_total(s_part, CH + ii, kk, P),
                      task == tid ? fbp : *out_at(args().F_beam, args().F_beam_c, i0 + ii, c0 + kk));
        }
    }
    }
    __syncthreads();   // every level's F_net is written before the heating reads it

    // heating of each layer from the net flux at its two interfaces (written above)
    const int NL = sub ? N / 2 : N;
    for (int task = tid; task < NL * K; task += W) {
        const int j = task / K, kk = task - j * K, cc = c0 + kk;
        if (cc >= C) continue;
        const long long o = (long long)j * C + cc;
        const double p0 = a.p[o], p1 = a.p[o + C];
        const double dp = p0 - p1;
        bool bad = !(dp > 0.0);
        if (sub) {
            const double pm = a.pc[o];
            bad = bad || !(p0 > pm && pm > p1);
        }
        if (bad) atomicOr(&s_flag[kk], (uint32_t)F_INVALID);
        const double qh = a.o.gravity * (a.F_net[o] - a.F_net[o + C]) / dp;
        a.heat[o] = qh;
        if (a.dTdt) a.dTdt[o] = qh / a.o.cp;
    }
    __syncthreads();
    for (int kk = tid; kk < K; kk += W) {
        const int cc = c0 + kk;
        if (cc >= C) continue;
        if (a.flags) a.flags[cc] = s_flag[kk];
        const uint32_t bad = status_bits(s_flag[kk]);
        if (status && bad) atomicOr(status, bad);
    }
}


// Workgroup of request r with first[r] <= g < first[r+1] (batched launches).
__device__ __forceinline__ int batch_slot(const int *first, int n, int g)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// MIXED: FP32 coefficients; IN32: FP32 storage of dtau, w0, g0 (mixed only)
template <bool MIXED, bool IN32 = false>
__global__ void __launch_bounds__(kMaxLaneThreads) k_solve_lane(const SolveArgs a)
{
    solve_tile_lane<MIXED, IN32>(a, blockIdx.x);
}

template <bool MIXED, bool IN32 = false>
__global__ void __launch_bounds__(kMaxLaneThreads)
k_solve_lane_batch(const SolveArgs *__restrict__ reqs, const int *__restrict__ first, int n)
{
    const int r = batch_slot(first, n, blockIdx.x);
    solve_tile_lane<MIXED, IN32>(reqs[r], blockIdx.x - first[r]);
}

template <bool MIXED, bool IN32 = false>
__global__ void __launch_bounds__(layer_max_threads(MIXED)) k_solve_layer(const SolveArgs a)
{
    solve_tile_layer<MIXED, IN32, true>(a, blockIdx.x, a.status, kernel_args(a));
}

template <bool MIXED, bool IN32 = false>
__global__ void __launch_bounds__(layer_max_threads(MIXED))
k_solve_layer_batch(const SolveArgs *__restrict__ reqs, const int *__restrict__ first, int n)
{
    const int r = batch_slot(first, n, blockIdx.x);
    solve_tile_layer<MIXED, IN32, true>(reqs[r], blockIdx.x - first[r], reqs[r].status, (ArgsK)(reqs + r));
}

int round64(int x) { return (x + 63) / 64 * 64; }

Geometry lane_geometry(int C, int NB, int K)
{
    Geometry g{};
    g.kernel = KERNEL_LANE;
    g.K = K > 0 ? K : std::max(1, 256 / NB);
    if (g.K > C) g.K = C;
    const int lanes = g.K * NB;
    if (lanes > kMaxLaneThreads) return Geometry{};
    g.threads = round64(lanes);
    g.blocks = (C + g.K - 1) / g.K;
    g.lanes = (long long)g.blocks * g.threads;
    const int ch = chunk_for(g.threads, g.K, NB);
    const size_t front = std::max((size_t)3 * ch * g.threads, (size_t)PC * g.K * (NB + 1));
    g.lds = front * 8 + (size_t)g.K * (ch + 1) * 8 + (size_t)(NB + 1) * 8 + (size_t)NB * 8 +
            (size_t)(NB + 2) * 4 + (size_t)g.K * 4;
    return g;
}

// Levels per chunk: the most work per barrier that fits LDS, with the items of
// a chunk (PC x lanes) in at most layer_items_per_thread rounds of the
// workgroup (each thread prefetches that many items of the next chunk).
// force_threads > 0: a workgroup of exactly that many threads (the serving
// worker's), else the kernel's bound for the precision.
Geometry layer_geometry(int C, int NB, int K, bool mixed, const DeviceLimits &dev, int NG,
                        int force_threads = 0)
{
    Geometry g{};
    g.kernel = KERNEL_LAYER;
    const int NBR = NG > 1 && NB % NG == 0 ? NB / NG : NB;   // bins (Planck edges NBR + 1)
    const int wmax = force_threads > 0 ? force_threads : layer_max_threads(mixed);
    if (K <= 0) {
        const int n_cu = dev.n_cu > 0 ? dev.n_cu : 256;
        K = (C + n_cu - 1) / n_cu;             // about one workgroup per compute unit
        K = std::max(1, std::min(K, wmax / NB));
    }
    if (K > C) K = C;
    const int T = K * NB;
    if (T > kMaxTileLanes) return Geometry{};
    if (T > wmax) return Geometry{};
    double best = -1.0;
    const int it = layer_items_per_thread(mixed);
    for (int pc = 1; pc <= 8; ++pc) {
        if (pc * T > it * wmax) break;
        const LpLayout lo = lp_layout(K, NB, NBR, pc, 1, mixed);
        if (lo.total > dev.lds) break;
        const int W = std::min(wmax, round64(pc * T));
        const int rounds = (pc * T + W - 1) / W;
        const double eff = double(pc * T) / (double(rounds) * W);
        const double score = eff * (1.0 - 0.15 / pc);
        if (score > best) {
            best = score;
            g.PC = pc;
            g.threads = W;
        }
    }
    if (best < 0.0) return Geometry{};
    // a multiple of four wavefronts, so that every SIMD of the compute unit
    // holds as many (the extra threads take no items, only edge integrals)
    g.threads = force_threads > 0 ? force_threads : std::min(wmax, (g.threads + 255) / 256 * 256);
    // interfaces per back-substitution pass: as many as fit in the threads'
    // staging registers and in the forward sweep's bytes, or in the device's
    // LDS for workgroups of 768 threads and more, which hold their compute
    // unit alone (register file) in either precision
    // (none with wavefront bin sums, which stage no records in LDS)
    const size_t front = lp_layout(K, NB, NBR, g.PC, 1, mixed).total;
    const size_t back_cap = g.threads >= 768 ? dev.lds : front;
    const bool ws = layer_wsum(K, NB, g.threads);
    int ch = 1;
    while (!ws && ch < 16 && lp_layout(K, NB, NBR, g.PC, ch + 1, mixed).total <= back_cap &&
           2 * (ch + 1) * T <= kBackUnits * g.threads)
        ++ch;
    g.CH = ch;
    g.K = K;
    g.blocks = (C + K - 1) / K;
    g.lanes = (long long)g.blocks * T;
    g.lds = lp_layout(K, NB, NBR, g.PC, g.CH, mixed, ws).total;
    return g;
}

}  // namespace

Geometry solve_geometry(int C, int N, int NB, int K, int kernel, int precision,
                        const DeviceLimits &dev, int NG)
{
    Geometry g = (kernel == KERNEL_LANE) ? lane_geometry(C, NB, K)
                                         : layer_geometry(C, NB, K, precision == 1, dev, NG);
    // the default tile of the layer kernel: narrower until its LDS fits
    if (g.threads == 0 && kernel != KERNEL_LANE && K <= 0) {
        const int n_cu = dev.n_cu > 0 ? dev.n_cu : 256;
        for (int k = std::min((C + n_cu - 1) / n_cu, layer_max_threads(precision == 1) / NB) - 1;
             k >= 1 && g.threads == 0; --k)
            g = layer_geometry(C, NB, k, precision == 1, dev, NG);
    }
    if (g.threads > 0)
        g.scratch = (size_t)N * (g.kernel == KERNEL_LANE ? 5 : 4) * (size_t)g.lanes * sizeof(double);
    return g;
}

Geometry worker_geometry(int C, int N, int NB, int precision, const DeviceLimits &dev, int NG)
{
    DeviceLimits d = dev;
    d.lds = dev.lds > kWorkerLdsReserve ? dev.lds - kWorkerLdsReserve : 0;
    const int n_cu = dev.n_cu > 0 ? dev.n_cu : 256;
    Geometry g{};
    for (int k = std::min((C + n_cu - 1) / n_cu, kWorkerThreads / NB); k >= 1 && g.threads == 0; --k)
        g = layer_geometry(C, NB, k, precision == 1, d, NG, kWorkerThreads);
    if (g.threads > 0) g.scratch = (size_t)N * 4 * (size_t)g.lanes * sizeof(double);
    return g;
}

namespace {

// Persistent serving worker.  Thread 0 of a workgroup claims the next published
// tile (compare-and-swap on the device-memory claim counter, below the
// host-published tail); the workgroup reads that request's arguments from
// pinned host memory, solves the tile with the layer kernel's body in the
// request's precision, and thread 0 stores the tile's completion word.  The
// wait for work is bounded: a workgroup exits after idle_polls polls without a
// tile, or once the host has set stop and nothing is left to claim, or at its
// next claim once another workgroup of the launch has idled out; so every
// launch ends, and the host launches the worker again for the work left.
__global__ void __launch_bounds__(kWorkerThreads) k_serve_worker(const WorkerArgs w)
{
    extern __shared__ double smem[];
    long long *s_claim = reinterpret_cast<long long *>(reinterpret_cast<char *>(smem) + w.lds_top);
    const int tid = threadIdx.x;
    unsigned int *const st = w.wg_status + blockIdx.x;
    // thread 0's one region per pass (a single region, so that no path of the
    // other threads can bypass it between two barriers): complete the previous
    // tile, then claim the next one
    long long prev = -1;
    for (;;) {
        if (tid == 0) {
            if (prev >= 0) {
                const unsigned bits = __hip_atomic_load(st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // the tile's outputs are visible before its completion word
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
                __hip_atomic_store(w.done + (prev & (long long)(w.ring_cap - 1)), 0x80000000u | bits,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            __hip_atomic_store(st, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            long long claim = -1;
            for (int it = 0;;) {
                // a lifetime that has begun to end takes no more tiles: a few
                // workgroups still on a tile would otherwise keep it alive and
                // serve later requests alone; its unclaimed tiles go to the next
                // lifetime, which the host launches once this one has ended
                if (__hip_atomic_load(w.exiting, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                const unsigned long long tail =
                    __hip_atomic_load(&w.q->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                unsigned long long h = __hip_atomic_load(w.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (h < tail) {
                    // a lost race means another workgroup claimed a tile: at most
                    // tail - h retries before the tiles run out
                    if (__hip_atomic_compare_exchange_strong(w.head, &h, h + 1ull, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        claim = (long long)h;
                        break;
                    }
                    continue;
                }
                if (__hip_atomic_load(&w.q->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) break;
                // idle: leave together, so that the host relaunches a whole worker
                // when work comes (workgroups still on a tile finish it first)
                if (++it >= w.idle_polls) {
                    __hip_atomic_store(w.exiting, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(32);
            }
            *s_claim = claim;
            prev = claim;
        }
        __syncthreads();
        // the claim as a wavefront-uniform value: every branch below is uniform
        const long long c = *s_claim;
        const int lo = __builtin_amdgcn_readfirstlane((int)(unsigned)(unsigned long long)c);
        const int hi = __builtin_amdgcn_readfirstlane((int)((unsigned long long)c >> 32));
        const long long claim = (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
        if (claim < 0) return;
        // the host's ring entry and request arguments, written before it published the tail
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        const int idx = (int)(claim & (long long)(w.ring_cap - 1));
        const unsigned long long e =
            __hip_atomic_load(reinterpret_cast<const unsigned long long *>(w.ring) + idx, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_SYSTEM);
        const int slot = __builtin_amdgcn_readfirstlane((int)(unsigned)e);
        const int tile = __builtin_amdgcn_readfirstlane((int)(unsigned)(e >> 32));
        // the request's arguments: one read across the bus into device memory
        // at this claim's ring position (not reused within a worker lifetime),
        // from where the tile's many loads of them hit the caches
        constexpr int kArgWords = (int)(sizeof(SlotArgs) / sizeof(unsigned long long));
        static_assert(kArgWords <= kWorkerThreads, "one word per thread");
        SlotArgs *ta = w.targs + idx;
        if (tid < kArgWords)
            reinterpret_cast<unsigned long long *>(ta)[tid] =
                reinterpret_cast<const unsigned long long *>(w.slots + slot)[tid];
        __syncthreads();
        const SlotArgs &sa = *ta;
        if (sa.mixed) solve_tile_layer<true, false, false>(sa.a, tile, st, nullptr);
        else solve_tile_layer<false, false, false>(sa.a, tile, st, nullptr);
        // every thread's outputs and condition bits of this tile precede thread
        // 0's completion word
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_worker(const WorkerArgs &w, const DeviceLimits &dev, hipStream_t s)
{
    const int grid = dev.n_cu > 0 ? dev.n_cu : 256;
    hipLaunchKernelGGL(k_serve_worker, dim3(grid), dim3(kWorkerThreads), dev.lds, s, w);
    return hipGetLastError();
}

hipError_t prepare_kernels(const DeviceLimits &dev)
{
    const int bytes = (int)dev.lds;
    const void *fns[] = {
        reinterpret_cast<const void *>(&k_solve_layer<false>),
        reinterpret_cast<const void *>(&k_solve_layer<true>),
        reinterpret_cast<const void *>(&k_solve_layer<true, true>),
        reinterpret_cast<const void *>(&k_solve_layer_batch<false>),
        reinterpret_cast<const void *>(&k_solve_layer_batch<true>),
        reinterpret_cast<const void *>(&k_solve_layer_batch<true, true>),
        reinterpret_cast<const void *>(&k_serve_worker)};
    for (const void *f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Kernel variant of a launch: FP64, mixed, or mixed with FP32 input storage.
enum Variant { V_FP64, V_MIXED, V_MIXED_IN32 };
static Variant variant(int precision, int in_f32)
{
    return precision != 1 ? V_FP64 : (in_f32 ? V_MIXED_IN32 : V_MIXED);
}

hipError_t launch_solve(const SolveArgs &a, const Geometry &g, int precision, hipStream_t s)
{
    SolveArgs b = a;
    b.K = g.K;
    b.PC = g.PC;
    b.CH = g.CH;
    b.L = g.lanes;
    const dim3 grid(g.blocks), block(g.threads);
    switch (variant(precision, a.in_f32)) {
    case V_FP64:
        if (g.kernel == KERNEL_LANE) hipLaunchKernelGGL(k_solve_lane<false>, grid, block, g.lds, s, b);
        else hipLaunchKernelGGL(k_solve_layer<false>, grid, block, g.lds, s, b);
        break;
    case V_MIXED:
        if (g.kernel == KERNEL_LANE) hipLaunchKernelGGL(k_solve_lane<true>, grid, block, g.lds, s, b);
        else hipLaunchKernelGGL(k_solve_layer<true>, grid, block, g.lds, s, b);
        break;
    case V_MIXED_IN32:
        if (g.kernel == KERNEL_LANE)
            hipLaunchKernelGGL((k_solve_lane<true, true>), grid, block, g.lds, s, b);
        else
            hipLaunchKernelGGL((k_solve_layer<true, true>), grid, block, g.lds, s, b);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_solve_batch(const SolveArgs *d_reqs, const int *d_first, int n, int total_blocks,
                              const Geometry &g, int precision, int in_f32, hipStream_t s)
{
    const dim3 grid(total_blocks), block(g.threads);
    const bool lane = g.kernel == KERNEL_LANE;
    switch (variant(precision, in_f32)) {
    case V_FP64:
        if (lane) hipLaunchKernelGGL(k_solve_lane_batch<false>, grid, block, g.lds, s, d_reqs, d_first, n);
        else hipLaunchKernelGGL(k_solve_layer_batch<false>, grid, block, g.lds, s, d_reqs, d_first, n);
        break;
    case V_MIXED:
        if (lane) hipLaunchKernelGGL(k_solve_lane_batch<true>, grid, block, g.lds, s, d_reqs, d_first, n);
        else hipLaunchKernelGGL(k_solve_layer_batch<true>, grid, block, g.lds, s, d_reqs, d_first, n);
        break;
    case V_MIXED_IN32:
        if (lane)
            hipLaunchKernelGGL((k_solve_lane_batch<true, true>), grid, block, g.lds, s, d_reqs, d_first, n);
        else
            hipLaunchKernelGGL((k_solve_layer_batch<true, true>), grid, block, g.lds, s, d_reqs, d_first,
                               n);
        break;
    }
    return hipGetLastError();
}

}  // namespace rtk

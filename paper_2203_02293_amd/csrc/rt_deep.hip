// rt_deep.hip -- layer-parallel solve for deep columns and few columns.
//
// Paper: Deitrick et al., "The THOR+HELIOS general circulation model"
// (arXiv 2203.02293): the same per-layer arithmetic as the other solve
// kernels (Section 2.2.1, Appendix B, `rt_physics.hpp`) and the same Thomas
// recurrence (Section 2.2.2); what changes is how the recurrence is
// scheduled.  The paper notes that many isothermal layers were too slow to
// use (Section 2.2.1); the other kernels walk a column's layers in one
// workgroup, so a grid of few columns leaves most of the chip idle.  Here each
// column's slabs are split into S segments from the TOA, one workgroup per
// (column, segment), and the recurrences are composed per segment:
//
//   k_deep_tau    per segment and lane: the sum of its optical depths.
//   k_deep_items  per segment: Planck, beam and the layer coefficients as
//                 (level, lane) and (layer, lane) items over all threads, and
//                 the segment's map of the elimination's (c, eps = 1 - c).
//   k_deep_eps    per lane, a tree scan over segments: c and eps at every
//                 segment top.
//   k_deep_elim   per segment: the elimination from there, with d at the
//                 segment top kept symbolic (d is affine in it); the records,
//                 and the segment's maps of d and of F_up.
//   k_deep_scan   per lane, tree scans over segments: d at every segment top,
//                 the BOA condition, F_up at every segment bottom.
//   k_deep_back   per segment: the back-substitution, bin sums and net flux of
//                 its levels.
//   k_deep_final  per (layer, column): heating rates.
//
// The elimination carries c_j and eps_j = 1 - c_j.  With A = 1 - r - t, one
// layer maps (c, eps) above it to (c', eps') below it as the 2x2 matrix
//   [ r(1-r) + t^2      r                          ]
//   [ A(1-r+t)          A(1-r+t) + r(1-r) + t^2    ]
// applied to (c, eps) and rescaled to c' + eps' = 1 (the rescaling divides by
// (1-r) c + eps = 1 - r c): every entry is non-negative, so a run of layers
// maps (c, eps) by the product of their matrices, formed without subtraction
// (rescaled by its largest entry), and c and eps both keep their relative
// precision however close to 0 or 1 they come.  Given c and eps,
// d' = S_dn + t (d + c S_up) / (1 - r c) is affine in d at the segment top,
// and F_up_{j+1} = G_j F_up_j + H_j is affine in F_up at the segment bottom;
// affine maps compose associatively, which the tree scans use.  Every step
// stays in FP64 except the coefficients of the mixed precision.
#include "rt_internal.hpp"
#include "rt_physics.hpp"

#include <algorithm>
#include <type_traits>

namespace rtk {
namespace {

// Work buffer of the deep path, L = C NB lanes, lane l = c NB + b:
//   coef [N][6][L]        t, r, 1-r, A, S_up, S_dn of every layer
//   rec  [N][6][L]        G, H0, Hs, c, d0, ds (H = H0 + Hs d_top, d = d0 + ds d_top)
//   fb   [N+1][L]         direct beam at every level
//   seg  [SG_COUNT][S][L] per segment (fields below)
//   lane [3][L]           F_BOA, F_up and F_dn at level 0
// The condition bits go straight to the flags output: k_deep_tau clears them,
// the later kernels OR into them (one atomic per workgroup).
enum SegField : int {
    SG_TAU = 0,                    // optical-depth sum of the segment's slabs
    SG_P00, SG_P01, SG_P10, SG_P11, // (c, eps) map of the segment
    SG_C_TOP, SG_EPS_TOP,          // c and eps at the segment top
    SG_D0, SG_DS,                  // d at the segment bottom = D0 + DS d_top
    SG_EPS_BOT, SG_C_BOT,          // eps and c at the segment bottom
    SG_GAM, SG_ETA0, SG_ETAS,      // F_up(top) = GAM F_up(bottom) + ETA0 + ETAS d_top
    SG_D_TOP, SG_FU_BOT,           // d at the top, F_up at the bottom
    SG_COUNT
};

struct DeepLayout {
    long long L;
    int S, Ls;
    double *coef, *rec, *fb, *seg, *lane;
};

__host__ __device__ __forceinline__ size_t deep_scratch_doubles(int C, int N, int NB, int S)
{
    const size_t L = (size_t)C * NB;
    (void)C;
    return (size_t)N * 12 * L + (size_t)(N + 1) * L + (size_t)SG_COUNT * S * L + 3 * L;
}

__device__ __forceinline__ DeepLayout deep_layout(const SolveArgs &a)
{
    DeepLayout d;
    d.L = (long long)a.C * a.NB;
    d.S = a.K;     // segments per column
    d.Ls = a.PC;   // slabs per segment
    d.coef = a.scratch;
    d.rec = d.coef + (long long)a.N * 6 * d.L;
    d.fb = d.rec + (long long)a.N * 6 * d.L;
    d.seg = d.fb + (long long)(a.N + 1) * d.L;
    d.lane = d.seg + (long long)SG_COUNT * d.S * d.L;
    return d;
}

__device__ __forceinline__ double &seg_at(const DeepLayout &d, int f, int s, long long l)
{
    return d.seg[((long long)f * d.S + s) * d.L + l];
}

// segment s: slabs top-1 .. bot, levels top .. bot (level j is interface j)
__device__ __forceinline__ void seg_range(const SolveArgs &a, const DeepLayout &d, int s, int &top,
                                          int &bot)
{
    top = a.N - s * d.Ls;
    bot = top - d.Ls;
    if (bot < 0) bot = 0;
}

// Temperature of level l and the bin-summed output slot of level l: on the
// sub-layer grid even levels are interfaces and odd levels layer centres.
__device__ __forceinline__ double T_level(const SolveArgs &a, int l, int cc)
{
    if (a.sub) return ((l & 1) ? a.Tc : a.T)[(long long)(l >> 1) * a.C + cc];
    return a.T[(long long)l * a.C + cc];
}

__device__ __forceinline__ double *out_level(const SolveArgs &a, double *iface, double *centre, int l,
                                             int cc)
{
    if (a.sub) return ((l & 1) ? centre : iface) + (long long)(l >> 1) * a.C + cc;
    return iface + (long long)l * a.C + cc;
}

// Workgroup size bound of the items kernel: the FP64 layer items need ~170
// VGPRs, which three wavefronts per SIMD hold; the FP32 items fit four.
__host__ __device__ constexpr int deep_items_max_threads(bool mixed) { return mixed ? 1024 : 768; }

// LDS of the items kernel for QL levels per chunk (byte offsets).
struct ItemsLds {
    size_t edge, B, Fb, tau, M, flag, total;
};

__host__ __device__ inline ItemsLds items_lds(int NB, int NBR, int QL, bool mixed)
{
    const size_t rs = mixed ? sizeof(float) : sizeof(double);
    auto up8 = [](size_t x) { return (x + 7) & ~(size_t)7; };
    ItemsLds o;
    o.edge = 0;                                                  // R [QL+1][NBR+1], row QL: T_int
    o.B = up8(o.edge + (size_t)(QL + 1) * (NBR + 1) * rs);       // R [QL+1][NB], row 0: carry
    o.Fb = up8(o.B + (size_t)(QL + 1) * NB * rs);                // double [QL+1][NB]
    o.tau = o.Fb + (size_t)(QL + 1) * NB * 8;                    // double [QL][NB]
    o.M = o.tau + (size_t)QL * NB * 8;                           // double [QL][4][NB]
    o.flag = o.M + (size_t)QL * 4 * NB * 8;                      // uint32
    o.total = o.flag + 8;
    return o;
}

// Workgroup size bound of the per-lane kernels: one thread per lane of a
// column, at most 768 lanes (bins x Gaussian points).
constexpr int kDeepLaneThreads = 768;

// Layers of one run of the elimination and levels of one pass of the
// back-substitution whose records a thread loads at once.
constexpr int kDeepRun = 8;

// Levels per pass of the back-substitution kernel: at most kDeepRun, its LDS
// within 64 KiB.
__host__ __device__ inline int back_chunk(int NB)
{
    const int c = (8192 - NB - 64) / (3 * NB);
    return c < 1 ? 1 : (c > kDeepRun ? kDeepRun : c);
}

__host__ __device__ inline size_t back_lds(int NB, int CH)
{
    return ((size_t)3 * CH * NB + NB + 3 * CH) * 8 + 8;
}

// OR the workgroup's condition bits (gathered in LDS word *s_flag) into the
// column's flags
__device__ __forceinline__ void flags_out(const SolveArgs &a, int c, const uint32_t *s_flag)
{
    if (threadIdx.x == 0 && a.flags && *s_flag) atomicOr(&a.flags[c], *s_flag);
    if (threadIdx.x == 0 && a.status && status_bits(*s_flag)) atomicOr(a.status, status_bits(*s_flag));
}

// Sum of p[k * stride] for k = 0 .. n-1 in that order, the loads issued in
// groups of 8 (adding 0 past the end is exact).
__device__ __forceinline__ double sum_strided(const double *p, long long stride, int n, int f32 = 0,
                                              long long i0 = 0)
{
    double acc = 0.0;
    for (int k0 = 0; k0 < n; k0 += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            v[q] = k0 + q < n ? ld_in(p, i0 + (long long)(k0 + q) * stride, f32) : 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += v[q];
    }
    return acc;
}

// ------------------------------------------------------------------ k_deep_tau
// Optical-depth sum of each segment and lane, from the top down; clears the
// flags.
__global__ void __launch_bounds__(kDeepLaneThreads) k_deep_tau(const SolveArgs a)
{
    const DeepLayout d = deep_layout(a);
    const int c = blockIdx.x / d.S, s = blockIdx.x - c * d.S, b = threadIdx.x;
    if (s == 0 && b == 0 && a.flags) a.flags[c] = 0u;
    if (b >= a.NB) return;
    int top, bot;
    seg_range(a, d, s, top, bot);
    const long long l = (long long)c * a.NB + b;
    seg_at(d, SG_TAU, s, l) =
        sum_strided(a.dtau, -d.L, top - bot, a.in_f32, (long long)(top - 1) * d.L + l);
}

// ---------------------------------------------------------------- k_deep_items
// The segment's levels top .. bot in chunks of QL = blockDim / NB levels:
//   1  per (level, lane) item thread: the slab above its level (dtau into LDS
//      for the optical-depth sums; dtau, w0, g0 kept for its layer item); the
//      Planck edge integrals of the chunk's levels (level, bin edge); on the
//      first chunk QL partial sums per lane of the segments above
//   2  per lane: the optical depth down the lane, in order
//   3  level items (level, lane): bin radiance and direct beam
//   4  layer items (layer, lane): coefficients into the work buffer, and each
//      layer's (c, eps) map into LDS
//   5  per lane: the maps composed into the segment's map
// Thread b < NB owns lane b's running optical depth and map.
template <bool MIXED>
__global__ void __launch_bounds__(deep_items_max_threads(MIXED)) k_deep_items(const SolveArgs a)
{
    using R = typename std::conditional<MIXED, float, double>::type;
    extern __shared__ double smem[];
    const DeepLayout d = deep_layout(a);
    const int c = blockIdx.x / d.S, s = blockIdx.x - c * d.S, tid = threadIdx.x, W = blockDim.x;
    const int NB = a.NB, NG = a.NG, NBR = NB / NG;
    const int QL = W / NB;
    const ItemsLds lo = items_lds(NB, NBR, QL, MIXED);
    char *base = reinterpret_cast<char *>(smem);
    R *s_edge = reinterpret_cast<R *>(base + lo.edge);
    R *s_B = reinterpret_cast<R *>(base + lo.B);
    double *s_Fb = reinterpret_cast<double *>(base + lo.Fb);
    double *s_tau = reinterpret_cast<double *>(base + lo.tau);
    double *s_M = reinterpret_cast<double *>(base + lo.M);
    uint32_t *s_flag = reinterpret_cast<uint32_t *>(base + lo.flag);
    int top, bot;
    seg_range(a, d, s, top, bot);
    const int nlev = top - bot + 1;
    const long long lc = (long long)c * NB;   // first lane of the column
    const double inv_eps2 = 1.0 / a.o.eps2;
    uint32_t fl = 0u;
    if (tid == 0) *s_flag = 0u;

    const double mu = a.mu[c];
    const bool day = mu > 0.0;
    const double inv_mu = day ? 1.0 / mu : 0.0;
    if (s == 0 && tid == 0) {
        if (!isfinite(mu)) fl |= F_INVALID;
        const double ti = a.Tint[c];
        if (!(ti >= 0.0) || !isfinite(ti)) fl |= F_INVALID;
    }
    const bool lane_thr = tid < NB;
    double tau = 0.0;
    double P00 = 1.0, P01 = 0.0, P10 = 0.0, P11 = 1.0;   // (c, eps) map of the layers so far
    // this thread's (level, lane) item of a chunk: level hi - iq, lane ib
    const int iq = tid / NB, ib = tid - iq * NB;

    auto bin_B = [&](const R *row, int rb, double Td) -> R {
        const R Tr = R(Td), T2 = Tr * Tr;
        R I = planck_combine<R>(row[rb], row[rb + 1]);
        if constexpr (MIXED) {
            const R iT = rcp(Tr);
            const R xb = a.c2_over_lam_f[rb] * iT, xa = a.c2_over_lam_f[rb + 1] * iT;
            if (planck_narrow(xa, xb)) {
                const double iTd = rcp(Td);
                I = planck_gl3(a.c2_over_lam[rb + 1] * iTd, a.c2_over_lam[rb] * iTd);
            }
        }
        return R(kPref) * T2 * T2 * I;
    };
    const bool boa = bot == 0;
    // inside the chunk loop the arguments (A) and the work-buffer layout (dl)
    // come from the kernel-argument segment, re-read in each chunk (ArgsK)
    ArgsK ap = kernel_args(a);

    for (int q0 = 0; q0 < nlev; q0 += QL) {
        opaque_args(ap);
        const SolveArgs &A = *(const SolveArgs *)ap;
        const DeepLayout dl = deep_layout(A);
        auto edge_val = [&](int e, double Tv) -> R { return planck_edge<R>(A.c2_over_lam[e] * rcp(Tv)); };
        const int hi = top - q0, n = min(QL, nlev - q0);
        // 1: the item's slab inputs (loads first, so they overlap the edge
        // integrals), the edge integrals, the partial sums above the segment
        const bool item = iq < n;
        const int ilev = hi - iq;
        const bool slab = item && ilev < top;   // slab ilev lies above level ilev
        double xdt = 0.0, xw = 0.0, xg = 0.0;
        if (slab) {
            const long long idx = (long long)ilev * dl.L + lc + ib;
            xdt = ld_in(A.dtau, idx, A.in_f32);
            xw = ld_in(A.w0, idx, A.in_f32);
            xg = ld_in(A.g0, idx, A.in_f32);
        }
        if (q0 == 0 && iq < QL)
            s_M[iq * NB + ib] = iq < s ? sum_strided(&seg_at(dl, SG_TAU, iq, lc + ib), (long long)QL * dl.L,
                                                     (s - iq + QL - 1) / QL)
                                       : 0.0;
        for (int e = tid; e < n * (NBR + 1); e += W) {
            const int q = e / (NBR + 1), k = e - q * (NBR + 1);
            const double Tv = T_level(A, hi - q, c);
            if (k == 0 && (!(Tv > 0.0) || !isfinite(Tv))) fl |= F_INVALID;
            s_edge[q * (NBR + 1) + k] = edge_val(k, Tv);
        }
        if (boa && q0 == 0)
            for (int e = tid; e <= NBR; e += W) s_edge[QL * (NBR + 1) + e] = edge_val(e, A.Tint[c]);
        if (item) s_tau[iq * NB + ib] = xdt;
        __syncthreads();
        // 2: optical depth down the lane: the segments above (first chunk),
        // then each slab in order from the top
        if (lane_thr) {
            if (q0 == 0)
                for (int g = 0; g < QL; ++g) tau += s_M[g * NB + tid];
            for (int q = 0; q < n; ++q) {
                tau += s_tau[q * NB + tid];
                s_tau[q * NB + tid] = tau;
            }
        }
        __syncthreads();
        // 3: level items
        for (int it = tid; it < n * NB; it += W) {
            const int q = it / NB, b = it - q * NB, lev = hi - q;
            const double Tv = T_level(A, lev, c);
            const R B = bin_B(s_edge + q * (NBR + 1), b / NG, Tv);
            double Fb = 0.0;
            if (day) {
                const double muF = mu * A.F_star[b / NG];
                Fb = lev == A.N ? muF : beam_at<MIXED>(muF, s_tau[q * NB + b], inv_mu);
            }
            s_B[(q + 1) * NB + b] = B;
            s_Fb[(q + 1) * NB + b] = Fb;
            if (lev > bot || boa) dl.fb[(long long)lev * dl.L + lc + b] = Fb;   // each level once
        }
        if (boa && q0 == 0 && lane_thr)
            dl.lane[lc + tid] = double(kPI) * double(bin_B(s_edge + QL * (NBR + 1), tid / NG, A.Tint[c]));
        __syncthreads();
        // 4: layer items, layer ilev between level ilev+1 (row iq) and level ilev (row iq+1)
        if (slab) {
            const int q = iq, b = ib;
            const Layer<R> Ly = layer_item<MIXED, R, MIXED>(xdt, xw, xg, day, mu, inv_mu,
                                                            s_Fb[q * NB + b], s_Fb[(q + 1) * NB + b],
                                                            s_B[(q + 1) * NB + b], s_B[q * NB + b], A.o,
                                                            inv_eps2, fl);
            // t and 1 - r from whichever of a value and its complement is the
            // smaller (both relatively exact): thin layers keep 1 - t and r to
            // the coefficients' relative precision, so FP32 rounding of t near
            // 1 does not accumulate along the column's transmission
            const double t = Ly.t < R(0.5) ? double(Ly.t) : 1.0 - double(Ly.omt);
            const double r = double(Ly.r);
            const double omr = Ly.r < R(0.5) ? 1.0 - r : double(Ly.omr);
            const double At = double(Ly.A);
            double *cp = dl.coef + (long long)ilev * 6 * dl.L + lc + b;
            cp[0] = t;
            cp[dl.L] = r;
            cp[2 * dl.L] = omr;
            cp[3 * dl.L] = At;
            cp[4 * dl.L] = double(Ly.Sup);
            cp[5 * dl.L] = double(Ly.Sdn);
            double *mp = s_M + q * 4 * NB + b;
            const double rt = r * omr + t * t, at = At * (omr + t);
            mp[0] = rt;
            mp[NB] = r;
            mp[2 * NB] = at;
            mp[3 * NB] = at + rt;
        }
        __syncthreads();
        // 5: compose the lane's maps (later layers on the left); carry the
        // chunk's last level to row 0 for the next chunk's first layer
        if (lane_thr) {
            for (int q = 0; q < n; ++q) {
                if (hi - q == top) continue;
                const double *mp = s_M + q * 4 * NB + tid;
                const double m00 = mp[0], m01 = mp[NB], m10 = mp[2 * NB], m11 = mp[3 * NB];
                const double q00 = m00 * P00 + m01 * P10, q01 = m00 * P01 + m01 * P11;
                const double q10 = m10 * P00 + m11 * P10, q11 = m10 * P01 + m11 * P11;
                const double mx = fmax(fmax(q00, q01), fmax(q10, q11));
                const double sc = mx > 0.0 ? rcp(mx) : 1.0;
                P00 = q00 * sc;
                P01 = q01 * sc;
                P10 = q10 * sc;
                P11 = q11 * sc;
            }
            s_B[tid] = s_B[n * NB + tid];
            s_Fb[tid] = s_Fb[n * NB + tid];
        }
        // the next chunk's phases 1 and 2 touch none of what phase 5 reads or
        // writes (s_M is rewritten only in phase 4, behind two barriers)
    }
    if (lane_thr) {
        const long long l = lc + tid;
        seg_at(d, SG_P00, s, l) = P00;
        seg_at(d, SG_P01, s, l) = P01;
        seg_at(d, SG_P10, s, l) = P10;
        seg_at(d, SG_P11, s, l) = P11;
    }
    if (fl) atomicOr(s_flag, fl);
    __syncthreads();
    flags_out(a, c, s_flag);
}

// ------------------------------------------------------------------- scans
// One group of Sp threads (a power of two >= S) per lane, 256 threads per
// workgroup; thread k of a group holds segment k.  Inclusive Hillis-Steele
// scans in LDS: at distance h, position k combines its value with position
// k - h's, its own (later) value applied last.

constexpr int kScanThreads = 256;

__device__ __forceinline__ int scan_width(int S)
{
    int p = 1;
    while (p < S) p <<= 1;
    return p;
}

// c and eps at every segment top, from the segments' maps (2x2, non-negative).
__global__ void __launch_bounds__(kScanThreads) k_deep_eps(const SolveArgs a)
{
    __shared__ double s_x[4][kScanThreads];
    const DeepLayout d = deep_layout(a);
    const int Sp = scan_width(d.S), tid = threadIdx.x, k = tid & (Sp - 1);
    const long long l = (long long)blockIdx.x * (kScanThreads / Sp) + tid / Sp;
    const bool act = l < d.L && k < d.S;
    double x00 = 1.0, x01 = 0.0, x10 = 0.0, x11 = 1.0;
    if (act) {
        x00 = seg_at(d, SG_P00, k, l);
        x01 = seg_at(d, SG_P01, k, l);
        x10 = seg_at(d, SG_P10, k, l);
        x11 = seg_at(d, SG_P11, k, l);
    }
    for (int h = 1; h < Sp; h <<= 1) {
        s_x[0][tid] = x00;
        s_x[1][tid] = x01;
        s_x[2][tid] = x10;
        s_x[3][tid] = x11;
        __syncthreads();
        if (k >= h) {
            const double p00 = s_x[0][tid - h], p01 = s_x[1][tid - h];
            const double p10 = s_x[2][tid - h], p11 = s_x[3][tid - h];
            const double q00 = x00 * p00 + x01 * p10, q01 = x00 * p01 + x01 * p11;
            const double q10 = x10 * p00 + x11 * p10, q11 = x10 * p01 + x11 * p11;
            const double mx = fmax(fmax(q00, q01), fmax(q10, q11));
            const double sc = mx > 0.0 ? rcp(mx) : 1.0;
            x00 = q00 * sc;
            x01 = q01 * sc;
            x10 = q10 * sc;
            x11 = q11 * sc;
        }
        __syncthreads();
    }
    s_x[0][tid] = x01;   // the maps applied to (c, eps) = (0, 1) at the TOA
    s_x[1][tid] = x11;
    __syncthreads();
    if (act) {
        double cv = 0.0, ev = 1.0;
        if (k > 0) {
            const double vc = s_x[0][tid - 1], ve = s_x[1][tid - 1], is = 1.0 / (vc + ve);
            cv = vc * is;
            ev = ve * is;
        }
        seg_at(d, SG_C_TOP, k, l) = cv;
        seg_at(d, SG_EPS_TOP, k, l) = ev;
    }
}

// d at every segment top (forward scan of d = D0 + DS d_top), the BOA
// condition, then F_up at every segment bottom (backward scan of
// F_up(top) = GAM F_up(bottom) + ETA0 + ETAS d_top).
__global__ void __launch_bounds__(kScanThreads) k_deep_scan(const SolveArgs a)
{
    __shared__ double s_x[2][kScanThreads];
    __shared__ double s_d[kScanThreads];
    __shared__ double s_f[kScanThreads];
    const DeepLayout d = deep_layout(a);
    const int S = d.S, Sp = scan_width(S), tid = threadIdx.x, k = tid & (Sp - 1);
    const int g0 = tid - k;   // first thread of the group
    const long long l = (long long)blockIdx.x * (kScanThreads / Sp) + tid / Sp;
    const bool lane_ok = l < d.L;
    const bool act = lane_ok && k < S;

    // affine maps x -> m x + v, composed later-after-earlier
    auto scan = [&](double &m, double &v) {
        for (int h = 1; h < Sp; h <<= 1) {
            s_x[0][tid] = m;
            s_x[1][tid] = v;
            __syncthreads();
            if (k >= h) {
                const double pm = s_x[0][tid - h], pv = s_x[1][tid - h];
                v = m * pv + v;
                m = m * pm;
            }
            __syncthreads();
        }
    };
    double m = 1.0, v = 0.0;
    if (act) {
        m = seg_at(d, SG_DS, k, l);
        v = seg_at(d, SG_D0, k, l);
    }
    scan(m, v);
    s_d[tid] = v;   // d at the bottom of segment k (segment 0's map is constant)
    __syncthreads();
    const double dtop = k == 0 ? 0.0 : s_d[tid - 1];
    if (act) seg_at(d, SG_D_TOP, k, l) = dtop;
    // BOA: F_up_0 - F_dn_0 = F_BOA + F_beam_0 with F_dn_0 = c_0 F_up_0 + d_0
    if (lane_ok && k == S - 1) {
        ElimState st;
        st.c = seg_at(d, SG_C_BOT, k, l);
        st.eps = seg_at(d, SG_EPS_BOT, k, l);
        st.d = v;
        double Fu, Fd;
        elim_boa(st, d.lane[l], d.fb[l], Fu, Fd);
        d.lane[d.L + l] = Fu;
        d.lane[2 * d.L + l] = Fd;
        s_f[g0] = Fu;
    }
    // backward: position k holds segment S-1-k (positions >= S: identity)
    const int sb = S - 1 - k;
    m = 1.0;
    v = 0.0;
    if (act) {
        m = seg_at(d, SG_GAM, sb, l);
        const double dt_sb = sb == 0 ? 0.0 : s_d[g0 + sb - 1];   // d at segment sb's top
        v = seg_at(d, SG_ETA0, sb, l) + seg_at(d, SG_ETAS, sb, l) * dt_sb;
    }
    __syncthreads();   // s_f of the group is written
    const double Fu0 = s_f[g0];
    scan(m, v);
    s_x[0][tid] = m;
    s_x[1][tid] = v;
    __syncthreads();
    if (act)
        seg_at(d, SG_FU_BOT, sb, l) = k == 0 ? Fu0 : s_x[0][tid - 1] * Fu0 + s_x[1][tid - 1];
}

// ----------------------------------------------------------------- k_deep_elim
__global__ void __launch_bounds__(kDeepLaneThreads) k_deep_elim(const SolveArgs a)
{
    const DeepLayout d = deep_layout(a);
    const int c = blockIdx.x / d.S, s = blockIdx.x - c * d.S, b = threadIdx.x;
    if (b >= a.NB) return;
    const long long l = (long long)c * a.NB + b;
    int top, bot;
    seg_range(a, d, s, top, bot);
    double eps = seg_at(d, SG_EPS_TOP, s, l);
    double cc = seg_at(d, SG_C_TOP, s, l);
    // d at the segment top: the TOA value on the first segment, else symbolic
    double d0 = s == 0 ? (a.Ftoa ? a.Ftoa[l] : 0.0) : 0.0, ds = s == 0 ? 0.0 : 1.0;
    double gam = 1.0, eta0 = 0.0, etas = 0.0;
    // runs of kDeepRun layers: the run's coefficients are loaded at once
    // (indices clamped into the segment, so every load is unconditional)
    for (int j0 = top - 1; j0 >= bot; j0 -= kDeepRun) {
        double ct[kDeepRun], cr[kDeepRun], co[kDeepRun], cA[kDeepRun], cu[kDeepRun], cd[kDeepRun];
#pragma unroll
        for (int q = 0; q < kDeepRun; ++q) {
            const double *cp = d.coef + (long long)max(j0 - q, bot) * 6 * d.L + l;
            ct[q] = cp[0];
            cr[q] = cp[d.L];
            co[q] = cp[2 * d.L];
            cA[q] = cp[3 * d.L];
            cu[q] = cp[4 * d.L];
            cd[q] = cp[5 * d.L];
        }
#pragma unroll
        for (int q = 0; q < kDeepRun; ++q) {
            const int j = j0 - q;
            if (j < bot) break;
            const double t = ct[q], r = cr[q], omr = co[q], A = cA[q], Sup = cu[q], Sdn = cd[q];
            const double inv = rcp(omr + r * eps);   // 1 / (1 - r c)
            const double G = t * inv, H0 = (r * d0 + Sup) * inv, Hs = r * ds * inv;
            double *rp = d.rec + (long long)j * 6 * d.L + l;
            rp[0] = G;
            rp[d.L] = H0;
            rp[2 * d.L] = Hs;
            rp[3 * d.L] = cc;
            rp[4 * d.L] = d0;
            rp[5 * d.L] = ds;
            eta0 += gam * H0;
            etas += gam * Hs;
            gam *= G;
            const double cn = r + t * t * cc * inv;
            const double en = (A * (omr + t) + eps * (r * omr + t * t)) * inv;
            const double dn0 = Sdn + t * (d0 + cc * Sup) * inv;
            const double dns = t * ds * inv;
            cc = cn;
            eps = en;
            d0 = dn0;
            ds = dns;
        }
    }
    seg_at(d, SG_D0, s, l) = d0;
    seg_at(d, SG_DS, s, l) = ds;
    seg_at(d, SG_EPS_BOT, s, l) = eps;
    seg_at(d, SG_C_BOT, s, l) = cc;
    seg_at(d, SG_GAM, s, l) = gam;
    seg_at(d, SG_ETA0, s, l) = eta0;
    seg_at(d, SG_ETAS, s, l) = etas;
}

// ----------------------------------------------------------------- k_deep_back
// Levels (bot, top] of the segment, and level 0 on the bottom segment, in
// passes of CH levels: per-lane fluxes into LDS, then the bin sums of each
// (quantity, level) by one thread over the lanes in order, then the net flux.
__global__ void __launch_bounds__(kDeepLaneThreads) k_deep_back(const SolveArgs a)
{
    extern __shared__ double smem[];
    const DeepLayout d = deep_layout(a);
    const int c = blockIdx.x / d.S, s = blockIdx.x - c * d.S, tid = threadIdx.x;
    const int NB = a.NB, NG = a.NG, NBR = NB / NG, CH = a.CH;
    const bool act = tid < NB;
    const int b = act ? tid : 0;
    const long long l = (long long)c * NB + b;
    int top, bot;
    seg_range(a, d, s, top, bot);
    double *s_v = smem;                    // [3][CH][NB]: F_up, F_dn, F_beam per lane
    double *s_w = s_v + 3 * CH * NB;       // [NB] quadrature weight of each lane
    double *s_sum = s_w + NB;              // [3][CH]
    uint32_t *s_flag = reinterpret_cast<uint32_t *>(s_sum + 3 * CH);
    for (int k = tid; k < NB; k += blockDim.x) s_w[k] = NG == 1 ? 1.0 : a.wg[k % NG];
    if (tid == 0) *s_flag = 0u;
    const double dtop = act ? seg_at(d, SG_D_TOP, s, l) : 0.0;
    double Fu = act ? seg_at(d, SG_FU_BOT, s, l) : 0.0, Fd = 0.0;
    const int lev0 = bot == 0 ? 0 : bot + 1;   // first level this segment writes
    for (int c0 = lev0; c0 <= top; c0 += CH) {
        const int nl = min(CH, top + 1 - c0);
        if (act) {
            // the pass's records (slab lev - 1 below level lev) and beam, loaded
            // at once (indices clamped, every load unconditional)
            double rG[kDeepRun], rH[kDeepRun], rc[kDeepRun], rd[kDeepRun], rb[kDeepRun];
#pragma unroll
            for (int q = 0; q < kDeepRun; ++q) {
                const int lev = min(c0 + q, top);
                const double *rp = d.rec + (long long)max(lev - 1, 0) * 6 * d.L + l;
                rG[q] = rp[0];
                rH[q] = rp[d.L] + rp[2 * d.L] * dtop;
                rc[q] = rp[3 * d.L];
                rd[q] = rp[4 * d.L] + rp[5 * d.L] * dtop;
                rb[q] = d.fb[(long long)lev * d.L + l];
            }
#pragma unroll
            for (int q = 0; q < kDeepRun; ++q) {
                if (q >= nl) break;
                const int lev = c0 + q;
                if (lev == 0) {
                    Fu = d.lane[d.L + l];
                    Fd = d.lane[2 * d.L + l];
                } else {
                    back_step(rG[q], rH[q], rc[q], rd[q], Fu, Fd);
                }
                const long long o = (long long)lev * d.L + l;
                if (a.F_up_bin) a.F_up_bin[o] = Fu;
                if (a.F_dn_bin) a.F_dn_bin[o] = Fd;
                if (lev == a.N && a.F_up_toa_bin && NG == 1) a.F_up_toa_bin[l] = Fu;
                s_v[(0 * CH + q) * NB + b] = Fu;
                s_v[(1 * CH + q) * NB + b] = Fd;
                s_v[(2 * CH + q) * NB + b] = rb[q];
            }
        }
        __syncthreads();
        for (int task = tid; task < 3 * nl; task += blockDim.x) {
            const int v = task / nl, q = task - v * nl;
            const double *row = s_v + (v * CH + q) * NB;
            double sum = 0.0;
            for (int k = 0; k < NB; ++k) sum += s_w[k] * row[k];
            double *out = v == 0 ? a.F_up : (v == 1 ? a.F_dn : a.F_beam);
            double *outc = v == 0 ? a.F_up_c : (v == 1 ? a.F_dn_c : a.F_beam_c);
            *out_level(a, out, outc, c0 + q, c) = sum;
            s_sum[v * CH + q] = sum;
        }
        // TOA spectrum per bin: the weighted sum over the bin's Gaussian points
        if (NG > 1 && a.F_up_toa_bin && c0 + nl - 1 == a.N) {
            for (int rb = tid; rb < NBR; rb += blockDim.x) {
                const double *row = s_v + (0 * CH + (a.N - c0)) * NB + rb * NG;
                double sum = 0.0;
                for (int g = 0; g < NG; ++g) sum += a.wg[g] * row[g];
                a.F_up_toa_bin[(long long)c * NBR + rb] = sum;
            }
        }
        __syncthreads();
        for (int q = tid; q < nl; q += blockDim.x) {
            const double fn = s_sum[q] - s_sum[CH + q] - s_sum[2 * CH + q];
            *out_level(a, a.F_net, a.F_net_c, c0 + q, c) = fn;
            if (!isfinite(fn)) atomicOr(s_flag, (uint32_t)F_NONFIN);
        }
        // the next pass writes s_v before its barrier and s_sum after it
    }
    __syncthreads();
    flags_out(a, c, s_flag);
}

// ---------------------------------------------------------------- k_deep_final
// Heating of each layer from the net flux at its two interfaces, one thread
// per (layer, column), and the pressure checks into the column's flags.
constexpr int kFinalThreads = 256;

__global__ void __launch_bounds__(kFinalThreads) k_deep_final(const SolveArgs a)
{
    const long long e = (long long)blockIdx.x * kFinalThreads + threadIdx.x;
    const int C = a.C, NL = a.sub ? a.N / 2 : a.N;
    if (e >= (long long)NL * C) return;
    const int j = (int)(e / C), c = (int)(e - (long long)j * C);
    const long long o = (long long)j * C + c;
    const double p0 = a.p[o], p1 = a.p[o + C];
    const double dp = p0 - p1;
    bool bad = !(dp > 0.0);
    if (a.sub) {
        const double pm = a.pc[o];
        bad = bad || !(p0 > pm && pm > p1);
    }
    if (bad && a.flags) atomicOr(&a.flags[c], (uint32_t)F_INVALID);
    if (bad && a.status) atomicOr(a.status, (uint32_t)F_INVALID);
    const double qh = a.o.gravity * (a.F_net[o] - a.F_net[o + C]) / dp;
    a.heat[o] = qh;
    if (a.dTdt) a.dTdt[o] = qh / a.o.cp;
}

// Workgroup size of the items kernel for segments of Ls slabs: (Ls + 1)
// levels x NB lanes (and x NBR + 1 edges) in one round if the bound allows.
__host__ __device__ inline int items_threads(int Ls, int NB, int NBR, bool mixed)
{
    const int lanes = (NB + 63) / 64 * 64;
    const int want = ((Ls + 1) * (NB > NBR + 1 ? NB : NBR + 1) + 63) / 64 * 64;
    const int w = want > lanes ? want : lanes;
    return w < deep_items_max_threads(mixed) ? w : deep_items_max_threads(mixed);
}

}  // namespace

Geometry deep_geometry(int C, int N, int NB, const DeviceLimits &dev)
{
    Geometry g{};
    g.kernel = KERNEL_DEEP;
    if (C < 1 || N < 1 || NB < 1 || NB > kDeepLaneThreads) return g;
    const int n_cu = dev.n_cu > 0 ? dev.n_cu : 256;
    // about two workgroups per compute unit, segments of at least 8 slabs,
    // at most 256 segments (one scan workgroup's width)
    int S = (2 * n_cu + C - 1) / C;
    S = std::max(1, std::min(S, kScanThreads));
    int Ls = (N + S - 1) / S;
    if (Ls < 8) Ls = std::min(8, N);
    S = (N + Ls - 1) / Ls;
    g.K = S;
    g.PC = Ls;
    g.CH = back_chunk(NB);
    g.threads = (NB + 63) / 64 * 64;
    g.blocks = C * S;
    g.lanes = (long long)C * NB;
    g.lds = back_lds(NB, g.CH);
    g.scratch = deep_scratch_doubles(C, N, NB, S) * sizeof(double);
    // the items kernel's LDS (largest with one bin per lane) within the device's
    for (int mixed = 0; mixed < 2; ++mixed) {
        const int wi = items_threads(Ls, NB, NB, mixed != 0);
        if (items_lds(NB, NB, wi / NB, mixed != 0).total > dev.lds) return Geometry{};
    }
    return g;
}

hipError_t prepare_deep_kernels(const DeviceLimits &dev)
{
    const int bytes = (int)dev.lds;
    hipError_t e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_deep_items<false>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess)
        return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_deep_items<true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_deep(const SolveArgs &a, const Geometry &g, int precision, hipStream_t s)
{
    SolveArgs b = a;
    b.K = g.K;    // segments per column
    b.PC = g.PC;  // slabs per segment
    b.CH = g.CH;  // levels per pass of the back-substitution
    b.L = g.lanes;
    const bool mixed = precision == 1;
    const int NB = a.NB, NBR = a.NB / a.NG;
    const int wi = items_threads(g.PC, NB, NBR, mixed);
    const size_t lds_items = items_lds(NB, NBR, wi / NB, mixed).total;
    int Sp = 1;
    while (Sp < g.K) Sp <<= 1;
    const unsigned scan_blocks = (unsigned)((g.lanes + kScanThreads / Sp - 1) / (kScanThreads / Sp));
    hipLaunchKernelGGL(k_deep_tau, dim3(g.blocks), dim3(g.threads), 0, s, b);
    if (mixed)
        hipLaunchKernelGGL(k_deep_items<true>, dim3(g.blocks), dim3(wi), lds_items, s, b);
    else
        hipLaunchKernelGGL(k_deep_items<false>, dim3(g.blocks), dim3(wi), lds_items, s, b);
    hipLaunchKernelGGL(k_deep_eps, dim3(scan_blocks), dim3(kScanThreads), 0, s, b);
    hipLaunchKernelGGL(k_deep_elim, dim3(g.blocks), dim3(g.threads), 0, s, b);
    hipLaunchKernelGGL(k_deep_scan, dim3(scan_blocks), dim3(kScanThreads), 0, s, b);
    hipLaunchKernelGGL(k_deep_back, dim3(g.blocks), dim3(g.threads), g.lds, s, b);
    const long long nlay = (long long)(a.sub ? a.N / 2 : a.N) * a.C;
    hipLaunchKernelGGL(k_deep_final, dim3((unsigned)((nlay + kFinalThreads - 1) / kFinalThreads)),
                       dim3(kFinalThreads), 0, s, b);
    return hipGetLastError();
}

}  // namespace rtk

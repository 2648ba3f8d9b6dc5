// rt_internal.hpp -- shared between the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rtk {

// Solver switches and constants copied into every launch.
struct Opts {
    int improved, noniso, e_clamp, pad_;
    double eps2, e_tau, g_guard, gravity, cp;
};

// The two solve kernels.
enum Kernel : int {
    KERNEL_AUTO = 0,
    KERNEL_LANE = 1,    // one thread per (column, bin) does everything for its lane
    KERNEL_LAYER = 2,   // Planck, beam and coefficients as (layer, column, bin) items
                        // shared by the workgroup; only the elimination is per lane
    KERNEL_DEEP = 3,    // a column's layers split into segments on separate
                        // workgroups, the recurrences composed per segment
};

// Everything one solve kernel needs (passed by value).
struct SolveArgs {
    int C, N, NB;              // columns, slabs (layers, or 2 x layers on the sub-layer grid), bins
    int K;                     // columns per workgroup
    int PC, CH;                // layer kernel: levels per chunk, interfaces per bin-sum pass
    int sub;                   // 1: sub-layer grid, N = 2 x layers slabs, levels interleaved
    int in_f32;                // 1: dtau, w0, g0 hold floats (ld_in)
    int NG;                    // Gaussian points per bin: NB = bins x NG lanes per column
    // resident tables of the handle
    const double *c2_over_lam; // [NB/NG+1] second radiation constant / edge
    const float *c2_over_lam_f;
    const double *F_star;      // [NB/NG]
    const double *wg;          // [NG] quadrature weights (NG > 1)
    // inputs
    const double *p, *T, *dtau, *w0, *g0, *mu, *Tint, *Ftoa;
    // outputs
    double *F_up, *F_dn, *F_beam, *F_net, *heat, *dTdt, *F_up_toa_bin, *F_up_bin, *F_dn_bin;
    uint32_t *flags;
    // serving: the request's status word, ORed with the condition bits that
    // fail a request (F_INVALID, F_EDOMAIN) of any column, or NULL
    uint32_t *status;
    // sub-layer grid: centre temperature/pressure [N/2][C], centre outputs [N/2][C]
    const double *Tc, *pc;
    double *F_up_c, *F_dn_c, *F_beam_c, *F_net_c;
    // work buffer of back-substitution records, [N][R][L] doubles with L lanes in
    // the grid (R = 5 for the lane kernel, 4 for the layer kernel)
    double *scratch;
    long long L;
    Opts o;
};

// Element i of a layer input (dtau, w0 or g0): stored as doubles, or as floats
// when f32 (the mixed path's FP32 storage); either way the FP64 number stored.
__host__ __device__ __forceinline__ double ld_in(const double *p, long long i, int f32)
{
    return f32 ? double(reinterpret_cast<const float *>(p)[i]) : p[i];
}

// A request's arguments in the constant address space: the kernel-argument
// segment of a single-request launch, or the descriptor table of a batched
// launch (written by the host before the launch); both stay unchanged while
// the kernel runs, so their fields may be read with scalar loads.  The solve
// kernels read the fields they use inside their loops through such a pointer,
// made opaque (opaque_args) at the top of each loop pass, so that each field
// is loaded with a scalar load where it is used: held for the whole kernel,
// the request's pointers outnumber the scalar registers, and the spilled ones
// come back through vector-lane moves of whole 16-register groups, which
// issue as vector instructions.
typedef const __attribute__((address_space(4))) SolveArgs *ArgsK;

// The arguments of a kernel whose only argument is the SolveArgs a: its
// kernel-argument segment (a at offset 0) on the GPU; a itself in the CPU
// builds of the kernels.
__host__ __device__ __forceinline__ ArgsK kernel_args(const SolveArgs &a)
{
#if defined(__HIP_DEVICE_COMPILE__)
    (void)a;
    return (ArgsK)__builtin_amdgcn_kernarg_segment_ptr();
#else
    return (ArgsK)&a;
#endif
}

// p, unchanged, as a value the compiler cannot follow past this point.
__host__ __device__ __forceinline__ void opaque_args(ArgsK &p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+s"(p));
#else
    (void)p;
#endif
}


// What the launch shape depends on besides the problem: the device.
struct DeviceLimits {
    int n_cu;          // compute units
    size_t lds;        // dynamic LDS bytes one workgroup may use
};

// Launch geometry of a solve for a problem shape.
struct Geometry {
    int kernel;     // KERNEL_LANE, KERNEL_LAYER or KERNEL_DEEP
    int K;          // columns per workgroup
    int PC, CH;     // layer kernel: levels per chunk, interfaces per bin-sum pass
    int threads;    // workgroup size (multiple of 64)
    int blocks;     // workgroups
    long long lanes;
    size_t lds;     // dynamic LDS bytes
    size_t scratch; // work-buffer bytes for N layers (set by solve_geometry)
};

constexpr int kMaxThreads = 1024;      // workgroup size bound of the solve kernels
constexpr int kMaxLaneThreads = 512;   // of the lane kernel
constexpr int kMaxTileLanes = 1024;    // (column, bin) lanes of one layer-kernel tile

// kernel: KERNEL_* (AUTO picks); K: columns per workgroup (0 = default).
// Returns threads = 0 when the shape cannot be launched (tile too large).
// NB: lanes per column (bins x NG Gaussian points).
Geometry solve_geometry(int C, int N, int NB, int K, int kernel, int precision,
                        const DeviceLimits &dev, int NG = 1);
hipError_t launch_solve(const SolveArgs &a, const Geometry &g, int precision, hipStream_t s);
// Layer-parallel path for deep columns (several launches on stream s): K =
// segments per column, PC = slabs per segment; scratch sized for it.
Geometry deep_geometry(int C, int N, int NB, const DeviceLimits &dev);
hipError_t launch_deep(const SolveArgs &a, const Geometry &g, int precision, hipStream_t s);
hipError_t prepare_deep_kernels(const DeviceLimits &dev);
// Several requests with the same kernel, tile, bins and precision in one launch:
// device arrays d_reqs[n] (K, PC, CH, L filled in) and d_first[n] (first
// workgroup of each).
hipError_t launch_solve_batch(const SolveArgs *d_reqs, const int *d_first, int n, int total_blocks,
                              const Geometry &g, int precision, int in_f32, hipStream_t s);
// Allow the kernels the device's full LDS per workgroup (once per device).
hipError_t prepare_kernels(const DeviceLimits &dev);

// ---------------------------------------------------------------- persistent serving
// A resident worker (one workgroup per compute unit, kWorkerThreads threads,
// the device's whole LDS) that takes layer-kernel tiles of any queued request
// from a ring the host fills, in either precision.  The ring, the request
// arguments and the completion words live in pinned host memory that the GPU
// reads and writes coherently; the claim counter lives in device memory.
constexpr int kWorkerThreads = 512;      // both precisions in one kernel: 256 VGPRs, 2 wavefronts per SIMD
constexpr size_t kWorkerLdsReserve = 256; // top of the LDS: the worker's own words

struct WorkTile {
    int slot;   // request slot
    int tile;   // workgroup tile of that request
};
// Arguments of one admitted request (a slot), as the worker reads them (with
// scalar loads, so each slot sits on cache lines of its own).
struct alignas(256) SlotArgs {
    SolveArgs a;
    int mixed, pad_[3];
};
static_assert(sizeof(SlotArgs) % 8 == 0, "the worker copies SlotArgs in 8-byte words");
// Host-written control words.
struct WorkQueueHost {
    unsigned long long tail;   // tiles published so far (stored with release order)
    unsigned int stop;         // 1: exit once no tile is left to claim
    unsigned int pad_;
};
struct WorkerArgs {
    WorkQueueHost *q;             // pinned host memory
    const WorkTile *ring;         // pinned host memory [ring_cap]
    const SlotArgs *slots;        // pinned host memory [n_slots]
    unsigned int *done;           // pinned host memory [ring_cap]: 0 = pending, else
                                  // 0x80000000 | condition bits of the finished tile
    SlotArgs *targs;              // device memory [ring_cap]: the claiming workgroup's
                                  // copy of the tile's request arguments (the tile
                                  // reads them there, not across the bus)
    unsigned long long *head;     // device memory: tiles claimed so far
    unsigned int *wg_status;      // device memory [grid]: condition bits of a tile
    unsigned int *exiting;        // device memory: set by the first workgroup that
                                  // idles out; the others then leave when idle too
    int ring_cap;                 // a power of two
    int idle_polls;               // polls without work before the worker exits
    int lds_top;                  // byte offset of the worker's own LDS words
    int pad_;
};
// Geometry of a request's tiles on the worker (the layer kernel at kWorkerThreads
// threads, within the LDS below the worker's reserve); threads = 0 if none fits.
Geometry worker_geometry(int C, int N, int NB, int precision, const DeviceLimits &dev, int NG);
hipError_t launch_worker(const WorkerArgs &w, const DeviceLimits &dev, hipStream_t s);

// Optical properties of the slabs from the opacity tables (one launch).
struct OpticsArgs {
    int C, S, NBG, NG;          // columns, slabs, lanes per column, Gaussian points per bin
    int sub, nT, nP, pad_;      // sub-layer grid; k-table grid sizes
    const double *temp, *log10p, *kappa;          // [nT], [nP], [nP][nT][NBG]
    const double *sig_gas, *sig_cl_abs, *sig_cl_scat, *g0_cl;   // [NB]; condensates pre-scaled by f
    double m_mean, gravity;
    const double *p, *T, *pc, *Tc;                // [N+1][C], [N][C]
    double *dtau, *w0, *g0;                       // [S][C][NBG]
};
hipError_t launch_optics(const OpticsArgs &a, hipStream_t s);
// Gas Rayleigh cross section (x_h2 H2 + x_he He, m^2 per molecule) averaged
// over [lam_lo, lam_hi] in wavenumber.
double rayleigh_bin_average(double lam_lo, double lam_hi, double x_h2, double x_he);

}  // namespace rtk

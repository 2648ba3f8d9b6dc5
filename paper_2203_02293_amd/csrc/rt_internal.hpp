// rt_internal.hpp -- shared between the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtk {

// Solver switches and constants copied into every launch.
struct Opts {
    int improved, noniso, e_clamp, pad_;
    double eps2, e_tau, g_guard, gravity, cp;
};

// Everything one solve kernel needs (passed by value).
struct SolveArgs {
    int C, N, NB;              // columns, layers, bins
    int K;                     // columns per workgroup
    // resident tables of the handle
    const double *c2_over_lam; // [NB+1] second radiation constant / edge
    const float *c2_over_lam_f;
    const double *F_star;      // [NB]
    // inputs
    const double *p, *T, *dtau, *w0, *g0, *mu, *Tint, *Ftoa;
    // outputs
    double *F_up, *F_dn, *F_beam, *F_net, *heat, *dTdt, *F_up_toa_bin, *F_up_bin, *F_dn_bin;
    uint32_t *flags;
    // work buffer: [N][5][L] doubles, L = lanes in the grid
    double *scratch;
    long long L;
    Opts o;
};

// Launch geometry of the solve kernel for a problem shape.
struct Geometry {
    int K;          // columns per workgroup
    int threads;    // workgroup size (multiple of 64)
    int blocks;     // workgroups
    long long lanes;
    size_t lds;     // dynamic LDS bytes
};

constexpr int kMaxThreads = 512;   // workgroup size bound of the solve kernel

int default_cols_per_block(int C, int NB);
Geometry solve_geometry(int C, int NB, int K);
size_t solve_scratch_bytes(int C, int N, int NB, int K);
hipError_t launch_solve(const SolveArgs &a, int precision, hipStream_t s);
// Several requests with the same tile width and bins in one launch: device arrays
// d_reqs[n] (with K and L filled in) and d_first[n] (first workgroup of each).
hipError_t launch_solve_batch(const SolveArgs *d_reqs, const int *d_first, int n, int total_blocks,
                              int threads, size_t lds, int precision, hipStream_t s);

}  // namespace rtk

/*
 * rt.h -- C-ABI of the MI355X improved two-stream radiative-transfer library.
 *
 * The library computes, for every atmospheric column and every k-table bin,
 * the improved two-stream fluxes of Deitrick et al., "The THOR+HELIOS general
 * circulation model" (arXiv 2203.02293): layer coefficients (Appendix B),
 * linear-in-tau Planck sources and the attenuated stellar beam (Section 2.2.1),
 * a Thomas-algorithm solve of the interface fluxes (Section 2.2.2), and the
 * bin sums into net fluxes and heating rates (Section 2.2.5: fluxes are
 * integrated over wavelength to obtain heating and cooling rates).
 *
 * Grid conventions (Section 2.2.1): interface i = 0 is the bottom of the
 * atmosphere (BOA) and i = N the top (TOA); layer j lies between interfaces j
 * (lower) and j+1 (upper).  Optical depth grows downward from the TOA.
 *
 * Memory: every array in rt_request is a DEVICE pointer owned by the caller,
 * 8-byte aligned, C-contiguous, in the layouts stated below.  The library owns
 * only its resident tables (bin edges, stellar flux, series coefficients) and
 * its own work buffers.  No function throws or aborts; all report an rt_status.
 * A handle is not thread-safe: use one handle per host thread or lock around it.
 */
#ifndef RT_MI355X_H
#define RT_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rt_status;
#define RT_OK          0   /* success (rt_poll: request finished)                */
#define RT_PENDING     1   /* rt_poll: request still queued or running           */
#define RT_EINVAL    (-1)  /* bad argument, shape or layout; nothing was launched */
#define RT_ENOMEM    (-2)  /* device allocation failed or request exceeds budget  */
#define RT_EDEVICE   (-3)  /* HIP runtime error (launch, copy, event)             */
#define RT_EDOMAIN   (-4)  /* strict E mode met E <= w0 (see flags)               */
#define RT_EBUSY     (-5)  /* serving queue full (max_inflight reached)           */
#define RT_ENOTFOUND (-6)  /* rt_poll/rt_wait on an unknown or retired ticket     */

/* precision of a solve */
#define RT_FP64  0   /* every step in FP64                                         */
#define RT_MIXED 1   /* FP32 coefficients, exponentials and Planck integrals; FP64
                        predicates, optical-depth sums and Thomas elimination     */

/* how the serving path (rt_submit) runs admitted requests (rt_config.serve_mode) */
#define RT_SERVE_BATCHED    0   /* requests admitted together share one launch
                                   (the default, and the faster design on MI355X
                                   at every load measured)                          */
#define RT_SERVE_PERSISTENT 1   /* a resident worker takes tiles of any admitted
                                   request as it frees up (layer-kernel requests
                                   with FP64 input storage; others run batched)    */

/* storage of the per-layer inputs dtau, w0, g0 (rt_request.input_dtype) */
#define RT_F64 0     /* doubles                                                     */
#define RT_F32 1     /* floats: RT_MIXED only (the FP64 path keeps its inputs exact) */

/* Solve kernels (same results to the precision's tolerance, different launch
 * shapes).  LANE: one thread per (column, bin) runs the whole sweep of its
 * lane.  LAYER: the Planck, beam and coefficient work of a tile is spread over
 * (layer, column, bin) items shared by the workgroup; only the FP64
 * elimination runs per lane.  DEEP: each column's layers are split into
 * segments on separate workgroups and the Thomas recurrence (Section 2.2.2)
 * is composed per segment and joined by scans over segments: for few, deep
 * columns; several launches on the stream (serving: a launch sequence of its
 * own per request), cols_per_block must be 0.  AUTO picks DEEP for at least 40
 * slabs with at most one column per 2 compute units, else LAYER. */
#define RT_KERNEL_AUTO  0
#define RT_KERNEL_LANE  1
#define RT_KERNEL_LAYER 2
#define RT_KERNEL_DEEP  3

/* per-column condition bits written to rt_request.flags */
#define RT_FLAG_GUARD    1u  /* G+- resonance guard (Section 2.2.1) replaced D by 2 mu_star */
#define RT_FLAG_ECLAMP   2u  /* E fit below 1 raised to 1 (e_clamp mode)                */
#define RT_FLAG_ETAU     4u  /* dtau < e_tau: layer treated as isothermal (Section 2.2.1) */
#define RT_FLAG_EDOMAIN  8u  /* strict mode: E <= w0, coefficients undefined            */
#define RT_FLAG_INVALID 16u  /* an input value is outside its documented domain         */
#define RT_FLAG_NONFIN  32u  /* a non-finite bin-summed output was produced             */

typedef struct rt_handle rt_handle;

/*
 * Static configuration, copied by rt_create (the host arrays may be freed
 * afterwards).  Defaults (rt_config_default) follow Table 3 of the paper.
 */
typedef struct {
    int32_t n_bins;               /* number of k-table bins NB, 1 <= NB <= 512       */
    int32_t improved;             /* 1: E from the fit of Section 2.2.4; 0: E = 1    */
    int32_t noniso;               /* 1: Planck linear in tau within a layer
                                     (non-isothermal layers); 0: isothermal layers,
                                     B = mean of the two interface values           */
    int32_t e_clamp;              /* 1: E = max(E_fit, 1) where the fit applies
                                     (no layer emits more than pi B); 0: strict,
                                     E <= w0 sets RT_FLAG_EDOMAIN                    */
    const double *lambda_edges;   /* HOST [NB+1] bin edges in metres, ascending      */
    const double *stellar_flux;   /* HOST [NB] stellar flux at TOA per bin, W m^-2,
                                     at normal incidence                             */
    double eps2;                  /* second Eddington coefficient of the beam (2/3)  */
    double e_tau;                 /* isothermal fallback threshold on dtau (1e-4)    */
    double g_guard;               /* |D| threshold of the G+- resonance guard (1e-5) */
    double gravity;               /* m s^-2 for the heating rate (47)                */
    double cp;                    /* J kg^-1 K^-1 for dT/dt (12436)                  */
    int64_t hbm_budget_bytes;     /* serving: cap on library-owned device memory used
                                     by in-flight requests (0: 8 GiB)                */
    int32_t max_inflight;         /* serving: max queued + running requests (0: 64)  */
    int32_t device;               /* HIP device ordinal                              */
    int32_t n_gauss;              /* k-distribution (Section 2.1.3): NG Gaussian
                                     points per bin (0 or 1: plain bins); each
                                     (bin, g) pair is solved with its bin's Planck
                                     function and stellar flux, and bin sums are
                                     sum_b sum_g w_g F.  NB * NG <= 768.           */
    int32_t serve_mode;           /* serving path: RT_SERVE_BATCHED (0) or
                                     RT_SERVE_PERSISTENT (see rt_submit)            */
    const double *gauss_weights;  /* HOST [NG] weights w_g > 0 (NULL if NG <= 1)   */
} rt_config;

/* Fill *cfg with the defaults (NB = 0 and NULL tables: the caller sets them). */
void rt_config_default(rt_config *cfg);

/*
 * Create a handle on cfg->device: validates cfg (RT_EINVAL), copies the bin
 * tables to the device and builds the resident series tables (RT_ENOMEM,
 * RT_EDEVICE).  *out is set only on RT_OK.
 */
rt_status rt_create(const rt_config *cfg, rt_handle **out);

/* Wait for the handle's own work, release everything it owns.  NULL is a no-op. */
rt_status rt_destroy(rt_handle *h);

/*
 * One solve.  Shapes: C = n_cols >= 1, N = n_layers in [1, 4096], NB from the
 * handle.  With NG > 1 Gaussian points per bin, every [..][NB] array below
 * except F_up_toa_bin has NB * NG entries instead, index b * NG + g, and
 * needs the layer kernel.  Inputs (device, read only):
 *   p_iface, T_iface  [N+1][C]   Pa, K; p strictly decreasing with i, T > 0
 *   dtau, w0, g0      [N][C][NB] layer optical depth (>= 0), single-scattering
 *                                albedo in [0,1], asymmetry in (-1,1); doubles,
 *                                or floats with input_dtype = RT_F32
 *   mu_star           [C]        cosine of the stellar zenith angle; <= 0: no beam
 *   T_int             [C]        interior temperature, F_BOA = pi B_b(T_int) (K, >= 0)
 *   F_toa             [C][NB]    diffuse downward flux at TOA (W m^-2) or NULL = 0
 * Outputs (device, written):
 *   F_up, F_dn, F_beam, F_net [N+1][C]  bin sums, W m^-2; F_net = F_up - F_dn - F_beam
 *   heating           [N][C]     W kg^-1, g (F_net_j - F_net_{j+1}) / (p_j - p_{j+1})
 *   dTdt              [N][C]     K s^-1 = heating / cp, or NULL
 *   F_up_toa_bin      [C][NB]    upward flux at TOA per bin (spectrum; the
 *                                weighted sum over its g-points), or NULL
 *   F_up_bin, F_dn_bin [N+1][C][NB] per-bin fluxes, or NULL
 *   flags             [C]        RT_FLAG_* bits per column, or NULL
 * Values outside their domain do not stop the solve: the column's outputs are
 * then unspecified and its flags carry RT_FLAG_INVALID.  On the stream path
 * (rt_solve_fluxes) such conditions are reported in flags only: the call
 * returns before the kernels run.  The serving path (rt_submit) also turns
 * them into the request's status (rt_poll/rt_wait).
 *
 * Sub-layer grid (non-isothermal layers split at their centres, Section 2.2.1
 * and the grid figure): set T_center (and p_center).  Each layer j is then two
 * slabs, lower (interface j to centre j) and upper (centre j to interface
 * j+1), each with its own optical properties and a Planck function linear in
 * optical depth between its two boundary levels:
 *   T_center, p_center [N][C]      centre temperature and pressure,
 *                                  p_iface[j] > p_center[j] > p_iface[j+1]
 *   dtau, w0, g0       [2N][C][NB] slab 2j = lower half of layer j, 2j+1 = upper
 *   F_up_center, F_dn_center, F_beam_center, F_net_center [N][C]  bin sums at
 *                                  the centres (all four required)
 *   F_up_bin, F_dn_bin [2N+1][C][NB] per-bin fluxes at all levels, interface j
 *                                  at level 2j and centre j at level 2j+1
 * Interface outputs and heating keep their shapes (heating per layer from the
 * interface net fluxes).  Needs the layer kernel (RT_KERNEL_LANE: RT_EINVAL).
 */
typedef struct {
    int32_t n_cols, n_layers;
    int32_t precision;            /* RT_FP64 or RT_MIXED */
    int32_t cols_per_block;       /* tile: columns per workgroup K (0 = the
                                     library's default for this shape); the tile
                                     must fit the kernel: K*NB <= 512 (lane
                                     kernel), K*NB <= 1024 and its LDS within the
                                     device's (layer kernel), else RT_EINVAL      */
    int32_t kernel;               /* RT_KERNEL_AUTO, _LANE, _LAYER or _DEEP */
    int32_t input_dtype;          /* storage of dtau, w0, g0: RT_F64 (doubles), or
                                     RT_F32 (floats; RT_MIXED only, else RT_EINVAL):
                                     half the bytes of the largest inputs.  Each
                                     value is used as the number it stores (the
                                     FP64 branch decisions see the float exactly) */
    const double *p_iface, *T_iface;
    const void *dtau, *w0, *g0;   /* double or float, as input_dtype says */
    const double *mu_star, *T_int;
    const double *F_toa;
    double *F_up, *F_dn, *F_beam, *F_net;
    double *heating, *dTdt;
    double *F_up_toa_bin;
    double *F_up_bin, *F_dn_bin;
    uint32_t *flags;
    /* sub-layer grid: NULL T_center = one slab per layer */
    const double *T_center, *p_center;
    double *F_up_center, *F_dn_center, *F_beam_center, *F_net_center;
} rt_request;

/*
 * Stream-ordered solve on hip_stream (a hipStream_t; NULL = the null stream).
 * Argument and shape errors return RT_EINVAL before any launch; a failed
 * launch returns RT_EDEVICE.  The buffers must stay valid until the stream's
 * work completes.  Solves on one handle share its work buffers: issue them on
 * one stream, or synchronise between streams.
 */
rt_status rt_solve_fluxes(rt_handle *h, const rt_request *req, void *hip_stream);

/*
 * rt_solve_fluxes for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same request, kernels and results, with the work buffer taken from a
 * fixed device array of the library (128 MiB per device, held from the
 * library's first use on a device until the process ends) instead of the
 * handle's, so the call makes no hipMalloc or hipFree and no other
 * allocating call.  The caller still owns every input and output buffer.
 * Errors: as rt_solve_fluxes, and RT_ENOMEM before any launch when the
 * request needs a larger work buffer than the array (rt_work_bytes gives the
 * need; at 2562 columns x 40 layers x 30 bins it is 98 MB).  Every call on a
 * device shares that one array and leaves its contents behind: calls on one
 * device that overlap (other streams, other handles, other threads) race;
 * issue them on one stream or synchronise between them.
 */
rt_status rt_solve_fluxes_noalloc(rt_handle *h, const rt_request *req, void *hip_stream);

/*
 * The kernel rt_solve_fluxes would run for req (RT_KERNEL_LANE, _LAYER or
 * _DEEP: AUTO resolved), checking req as rt_solve_fluxes does but launching
 * nothing; RT_EINVAL (negative) on a bad request.
 */
int32_t rt_request_kernel(rt_handle *h, const rt_request *req);

/*
 * Serving path: enqueue a request and return at once with *ticket.  The
 * library admits queued requests onto the device in arrival order when its
 * memory budget allows; requests of the same kernel, precision and tile width
 * that are admitted together run as one batched launch (each workgroup finds
 * its request and column tile in a descriptor table), up to 64 per launch; a
 * request on the deep kernel runs as its own launch sequence; 16 batches in
 * flight on 4 library-owned streams.  Results equal those of rt_solve_fluxes
 * (same request) bit for bit.  With serve_mode = RT_SERVE_PERSISTENT, a
 * request that runs on the layer kernel with FP64 input storage goes instead
 * to a resident worker (one workgroup per compute unit, launched by the
 * library when work is waiting and ending by itself a fraction of a millisecond after
 * the last tile): the request's tiles are published to a ring in pinned host
 * memory as soon as a request slot (4096 per worker lifetime), ring space
 * (65536 tiles) and budget memory are free, and any idle workgroup takes the
 * next tile, so tiles of different requests and precisions share the device
 * without a launch per batch.  Its tile is the worker's (512 threads, the
 * LDS less 256 bytes), so its results equal those of the
 * same request on the worker, alone or in any mix, bit for bit, and those of
 * rt_solve_fluxes to the precision's tolerance.  Requests retire in any order.  The inputs must
 * be complete on the device before the call (the library's streams do not wait
 * on the caller's), and the request's buffers must stay valid, and must not be
 * touched, until rt_poll/rt_wait returns something other than RT_PENDING.  Errors:
 * RT_EINVAL (bad request), RT_EBUSY (max_inflight reached), RT_ENOMEM (the
 * request alone exceeds the memory budget, or the budget's device memory
 * could not be allocated; the handle stays usable).
 */
rt_status rt_submit(rt_handle *h, const rt_request *req, uint64_t *ticket);

/*
 * Non-blocking: RT_PENDING while the request is queued or running; once it
 * has finished (the ticket then retires): RT_OK, or RT_EDOMAIN if a column
 * met E <= w0 in strict mode (e_clamp = 0, Section 2.2.4), else RT_EINVAL if
 * an input value was outside its domain (the columns' flags say which), or
 * RT_EDEVICE if its launch failed.  The outputs are written in every case.
 * RT_ENOTFOUND for an unknown or retired ticket.
 */
rt_status rt_poll(rt_handle *h, uint64_t ticket);

/* Blocking variant of rt_poll (same results). */
rt_status rt_wait(rt_handle *h, uint64_t ticket);

/*
 * Optical properties: the step before the solve (Sections 2.1.3 and 2.2.3,
 * Appendix C).  dtau, w0 and g0 of every slab from
 *   - a pre-mixed k-table: gas absorption opacity per unit mass kappa for
 *     every (bin, Gaussian point), interpolated bilinearly in T and log10 p
 *     (held at the table's edge outside it);
 *   - gas Rayleigh scattering per molecule, x_H2 sigma_H2 + x_He sigma_He with
 *     the printed cross sections, averaged over each bin in wavenumber;
 *   - condensates with per-particle cross sections, f_cloud per gas molecule;
 * mixed as extinction = sigma_scat,gas + kappa m + f (sigma_abs,cl +
 * sigma_scat,cl), w0 = (sigma_scat,gas + f sigma_scat,cl) / extinction,
 * g0 = f sigma_scat,cl g0,cl / (sigma_scat,gas + f sigma_scat,cl) (0 without
 * scattering), and dtau = extinction / m x (pressure thickness) / gravity.
 * One slab per layer takes the properties at the layer centre; on the
 * sub-layer grid each sub-layer takes the arithmetic mean of the properties
 * at its two levels (Section 2.2.1).
 */
typedef struct {
    int32_t n_temp, n_press;      /* table grid, each in [2, 1024]                  */
    const double *temp;           /* HOST [n_temp] K, strictly ascending            */
    const double *log10p;         /* HOST [n_press] log10(p / Pa), strictly ascending */
    const double *kappa;          /* HOST [n_press][n_temp][NB*NG] m^2 kg^-1, >= 0  */
    const double *cloud_abs;      /* HOST [NB] m^2 per particle, or NULL (no clouds;
                                     then cloud_scat and cloud_g0 are NULL too)     */
    const double *cloud_scat;     /* HOST [NB] m^2 per particle                     */
    const double *cloud_g0;       /* HOST [NB] asymmetry of the condensates         */
    double f_cloud;               /* condensate-to-gas number ratio (1e-17), >= 0   */
    double m_mean;                /* mean molecular mass, kg (2.34 amu), > 0        */
    double x_h2, x_he;            /* volume mixing ratios for Rayleigh scattering   */
} rt_opacities;

/* Copy the tables to the device (replacing earlier ones).  RT_EINVAL on bad
 * values or sizes, RT_ENOMEM / RT_EDEVICE on device failures.  Waits for the
 * handle's work first. */
rt_status rt_set_opacities(rt_handle *h, const rt_opacities *op);

typedef struct {
    int32_t n_cols, n_layers;     /* C >= 1, N in [1, 4096]                         */
    int32_t sublayer;             /* 0: one slab per layer; 1: sub-layer grid       */
    int32_t reserved;             /* must be 0                                      */
    const double *p_iface, *T_iface;    /* DEVICE [N+1][C] Pa, K                    */
    const double *p_center, *T_center;  /* DEVICE [N][C] Pa, K                      */
    double *dtau, *w0, *g0;       /* DEVICE out [S][C][NB*NG], S = N or 2N slabs    */
} rt_optics_request;

/* Stream-ordered; RT_EINVAL without opacities set or on bad arguments. */
rt_status rt_optical_properties(rt_handle *h, const rt_optics_request *req, void *hip_stream);

/*
 * Device bytes of work buffer one solve of this shape needs with the default
 * choices (RT_KERNEL_AUTO, default tile, no sub-layer grid): what the serving
 * path reserves from its budget for such a request; -1 on bad arguments.
 */
int64_t rt_work_bytes(const rt_handle *h, int32_t n_cols, int32_t n_layers);

/* Latest error message of the handle (never NULL; "" if none). */
const char *rt_last_error(const rt_handle *h);

/* Static description of a status code. */
const char *rt_status_string(rt_status s);

#ifdef __cplusplus
}
#endif
#endif

// rt_api.hip -- host side of the C-ABI declared in include/rt.h.
//
// Validation, resident tables, work buffers and launches of the solve kernel
// (stream-ordered path), plus the serving path: a request queue, admission by
// device-memory footprint against a fixed arena, concurrent execution on a
// small pool of streams, and completion tracking with events.
#include "rt.h"
#include "rt_internal.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <chrono>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

namespace {

constexpr double kH = 6.62607015e-34, kC = 299792458.0, kKB = 1.380649e-23;
constexpr int kMaxBins = 512;
constexpr int kMaxBinPoints = 768;   // bins x Gaussian points: lanes of one column
constexpr int kMaxLayers = 4096;
// AUTO takes the deep kernel from this many slabs, for at most one column per
// this many compute units (measured crossover: 128 columns at 40 to 400 layers
// on 256 compute units)
constexpr int kDeepMinSlabs = 40;
constexpr int kDeepColsPerCu = 2;
constexpr int kStreams = 4;
constexpr size_t kAlign = 256;

// First-fit sub-allocator over one device arena (serving work buffers).
struct Arena {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length

    void reset(char *p, size_t n)
    {
        base = p;
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t *off)
    {
        n = (n + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                size_t rest = it->second - n, o = it->first + n;
                free_.erase(it);
                if (rest) free_[o] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (n + kAlign - 1) / kAlign * kAlign;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Job {
    uint64_t ticket;
    rt_request req;
    rtk::Geometry g;           // launch shape of this request
    size_t bytes = 0, off = 0; // reservation in the serving arena
};

// Persistent serving: ring of published tiles, ring of request slots, and the
// worker's idle bound (polls of about 1-3 us each before it exits).  The
// worker reads a slot with scalar loads, whose cache the host cannot
// invalidate: so a slot is never rewritten during one worker lifetime (slots
// are taken in sequence; a request whose slot was last used by a request
// still running at the worker's launch waits for the next lifetime).
constexpr int kRingCap = 1 << 16;
constexpr int kSlotRing = 4096;
constexpr int kIdlePolls = 50;

// A request admitted to the persistent worker: its slot and its tiles
// [first, first + ntiles) of the ring; tiles before `seen` have completed.
struct PJob {
    Job j;
    uint64_t seq = 0;   // slot sequence number (slot = seq % kSlotRing)
    int slot = 0;
    uint64_t first = 0;
    int ntiles = 0, seen = 0;
    uint32_t bits = 0;
};

constexpr int kMaxBatch = 64;  // requests per batched launch
constexpr int kSlots = 16;     // batches in flight

// One batched launch in flight: its requests, descriptor buffers and event.
struct Batch {
    bool busy = false;
    std::vector<Job> jobs;
    rtk::SolveArgs *h_args = nullptr;   // pinned host staging
    int *h_first = nullptr;
    rtk::SolveArgs *d_args = nullptr;   // device copy read by the kernel
    int *d_first = nullptr;
    uint32_t *d_status = nullptr;       // per request: condition bits that fail it
    uint32_t *h_status = nullptr;       // pinned copy, read once the batch is done
    hipEvent_t done = nullptr;
    int stream = 0;
};

// Work buffer of rt_solve_fluxes_noalloc: a file-scope device array, so that
// entry point allocates nothing.  Each device the library runs on holds its
// own copy from the first use of the library on it until the process ends.
// In host code the array's name is not a device address: its address on a
// device comes from hipGetSymbolAddress (static_scratch below).
constexpr size_t kStaticScratchBytes = size_t(128) << 20;   // 128 MiB
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
double *g_static_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (which must be current), looked
// up once per device; nullptr if the lookup fails.
double *static_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_static_ptr[dev] = static_cast<double *>(p);
    }
    return g_static_ptr[dev];
}

}  // namespace

struct rt_handle {
    rt_config cfg{};
    int NB = 0;          // bins
    int NG = 1;          // Gaussian points per bin
    int NBG = 0;         // lanes per column, NB * NG
    rtk::DeviceLimits dev{};
    double *d_gw = nullptr;
    std::vector<double> lam;   // bin edges, m (host copy)
    // opacity tables (rt_set_opacities)
    bool have_opac = false;
    int opac_nT = 0, opac_nP = 0;
    double opac_m = 0.0;
    double *d_opac = nullptr;   // temp[nT], log10p[nP], kappa[nP][nT][NBG], then [4][NB] per-bin terms
    double *d_c2lam = nullptr;
    float *d_c2lam_f = nullptr;
    double *d_fstar = nullptr;
    double *d_scratch = nullptr;
    size_t scratch_bytes = 0;
    double *static_ws = nullptr;   // this device's `scratch` (rt_solve_fluxes_noalloc)
    std::string err;
    // serving
    hipStream_t streams[kStreams] = {};
    int next_stream = 0;
    void *arena_mem = nullptr;
    Arena arena;
    uint64_t next_ticket = 1;
    std::deque<Job> queued;
    Batch slots[kSlots];
    std::map<uint64_t, int> running;          // ticket -> batch slot
    std::map<uint64_t, rt_status> finished;   // retired on first poll
    // persistent serving (serve_mode RT_SERVE_PERSISTENT)
    rtk::WorkQueueHost *wq = nullptr;         // pinned host memory: control words
    rtk::WorkTile *wring = nullptr;           // [kRingCap]
    rtk::SlotArgs *wslots = nullptr;          // [kSlotRing]
    unsigned int *wdone = nullptr;            // [kRingCap] completion words
    rtk::WorkerArgs wargs{};                  // device-side view of the above
    rtk::SlotArgs *d_targs = nullptr;         // device: [kRingCap] argument copies
    unsigned long long *d_head = nullptr;     // device: tiles claimed
    unsigned int *d_wgst = nullptr;           // device: per-workgroup condition bits
    unsigned int *d_exiting = nullptr;        // device: the worker is idling out
    hipStream_t wstream = nullptr;
    hipEvent_t wevent = nullptr;              // recorded after each worker launch
    bool wlaunched = false;
    bool wbroken = false;                     // a worker launch failed: requests go batched
    uint64_t wpublished = 0;                  // tiles published
    uint64_t wseq = 0;                        // slots taken
    uint64_t wgen = 0;                        // oldest slot the running worker may read
    uint64_t wlife0 = 0;                      // first ring position it may claim
    std::deque<Job> pqueued;                  // waiting for the worker
    std::map<uint64_t, PJob> prunning;        // admitted to the worker
};

// Device allocation that leaves no error behind: a failed hipMalloc also sets
// the runtime's last-error state, which the caller's next unrelated HIP call
// (or the framework around the library) would otherwise report as its own.
static bool dev_alloc(void **p, size_t bytes)
{
    if (hipMalloc(p, bytes) == hipSuccess) return true;
    (void)hipGetLastError();
    *p = nullptr;
    return false;
}

static bool host_alloc(void **p, size_t bytes)
{
    if (hipHostMalloc(p, bytes) == hipSuccess) return true;
    (void)hipGetLastError();
    *p = nullptr;
    return false;
}

static rt_status fail(rt_handle *h, rt_status s, const char *fmt, ...)
{
    if (h) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        h->err = buf;
    }
    return s;
}

static rt_status hip_fail(rt_handle *h, hipError_t e, const char *what)
{
    return fail(h, RT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

extern "C" void rt_config_default(rt_config *c)
{
    if (!c) return;
    std::memset(c, 0, sizeof *c);
    c->improved = 1;
    c->noniso = 1;
    c->e_clamp = 1;
    c->eps2 = 2.0 / 3.0;
    c->e_tau = 1e-4;
    c->g_guard = 1e-5;
    c->gravity = 47.0;
    c->cp = 12436.0;
    c->hbm_budget_bytes = 0;
    c->max_inflight = 0;
    c->device = 0;
}

extern "C" const char *rt_status_string(rt_status s)
{
    switch (s) {
    case RT_OK: return "ok";
    case RT_PENDING: return "pending";
    case RT_EINVAL: return "invalid argument";
    case RT_ENOMEM: return "out of device memory or over budget";
    case RT_EDEVICE: return "HIP runtime error";
    case RT_EDOMAIN: return "E <= w0 in strict mode";
    case RT_EBUSY: return "serving queue full";
    case RT_ENOTFOUND: return "unknown ticket";
    default: return "unknown status";
    }
}

// AUTO on a stream-ordered solve: the deep kernel where the layer kernel's
// workgroups (about one per column up to one per compute unit) would leave
// most of the chip idle for a long sweep.
static bool prefer_deep(const rt_handle *h, int C, int N)
{
    return N >= kDeepMinSlabs && (long long)C * kDeepColsPerCu <= h->dev.n_cu;
}

extern "C" int64_t rt_work_bytes(const rt_handle *h, int32_t n_cols, int32_t n_layers)
{
    if (!h || n_cols < 1 || n_layers < 1 || n_layers > kMaxLayers) return -1;
    const rtk::Geometry g =
        prefer_deep(h, n_cols, n_layers)
            ? rtk::deep_geometry(n_cols, n_layers, h->NBG, h->dev)
            : rtk::solve_geometry(n_cols, n_layers, h->NBG, 0, rtk::KERNEL_AUTO, RT_FP64, h->dev,
                                  h->NG);
    return g.threads > 0 ? (int64_t)g.scratch : -1;
}

extern "C" const char *rt_last_error(const rt_handle *h)
{
    return h ? h->err.c_str() : "null handle";
}

extern "C" rt_status rt_create(const rt_config *cfg, rt_handle **out)
{
    if (!cfg || !out) return RT_EINVAL;
    const int NB = cfg->n_bins;
    if (NB < 1 || NB > kMaxBins || !cfg->lambda_edges || !cfg->stellar_flux) return RT_EINVAL;
    for (int e = 0; e <= NB; ++e) {
        double l = cfg->lambda_edges[e];
        if (!(l > 0.0) || !std::isfinite(l)) return RT_EINVAL;
        if (e > 0 && !(l > cfg->lambda_edges[e - 1])) return RT_EINVAL;
    }
    for (int b = 0; b < NB; ++b)
        if (!(cfg->stellar_flux[b] >= 0.0) || !std::isfinite(cfg->stellar_flux[b])) return RT_EINVAL;
    if (!(cfg->eps2 > 0.0) || !(cfg->e_tau >= 0.0) || !(cfg->g_guard >= 0.0) ||
        !(cfg->gravity > 0.0) || !(cfg->cp > 0.0) || cfg->hbm_budget_bytes < 0 ||
        cfg->max_inflight < 0 || cfg->n_gauss < 0 ||
        (cfg->serve_mode != RT_SERVE_BATCHED && cfg->serve_mode != RT_SERVE_PERSISTENT))
        return RT_EINVAL;
    const int NG = cfg->n_gauss > 1 ? cfg->n_gauss : 1;
    if ((long long)NB * NG > kMaxBinPoints) return RT_EINVAL;
    if (NG > 1) {
        if (!cfg->gauss_weights) return RT_EINVAL;
        for (int g = 0; g < NG; ++g)
            if (!(cfg->gauss_weights[g] > 0.0) || !std::isfinite(cfg->gauss_weights[g]))
                return RT_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev)
        return RT_EDEVICE;
    if (hipSetDevice(cfg->device) != hipSuccess) return RT_EDEVICE;

    rt_handle *h = new (std::nothrow) rt_handle();
    if (!h) return RT_ENOMEM;
    h->cfg = *cfg;
    h->cfg.lambda_edges = nullptr;
    h->cfg.stellar_flux = nullptr;
    h->cfg.gauss_weights = nullptr;
    if (h->cfg.hbm_budget_bytes == 0) h->cfg.hbm_budget_bytes = 8ll << 30;
    if (h->cfg.max_inflight == 0) h->cfg.max_inflight = 64;
    h->NB = NB;
    h->lam.assign(cfg->lambda_edges, cfg->lambda_edges + NB + 1);
    h->NG = NG;
    h->NBG = NB * NG;
    {
        int n_cu = 0, lds = 0;
        if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, cfg->device) !=
                hipSuccess ||
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, cfg->device) !=
                hipSuccess) {
            delete h;
            return RT_EDEVICE;
        }
        h->dev.n_cu = n_cu;
        h->dev.lds = (size_t)lds;
        if (rtk::prepare_kernels(h->dev) != hipSuccess ||
            rtk::prepare_deep_kernels(h->dev) != hipSuccess) {
            delete h;
            return RT_EDEVICE;
        }
        // the allocation-free path's work buffer on this device (current here)
        h->static_ws = static_scratch(cfg->device);
        if (!h->static_ws) {
            delete h;
            return RT_EDEVICE;
        }
    }

    std::vector<double> c2(NB + 1);
    std::vector<float> c2f(NB + 1);
    const double c2rad = kH * kC / kKB;
    for (int e = 0; e <= NB; ++e) {
        c2[e] = c2rad / cfg->lambda_edges[e];
        c2f[e] = float(c2[e]);
    }
    if (!dev_alloc((void **)&h->d_c2lam, sizeof(double) * (NB + 1)) ||
        !dev_alloc((void **)&h->d_c2lam_f, sizeof(float) * (NB + 1)) ||
        !dev_alloc((void **)&h->d_fstar, sizeof(double) * NB) ||
        !dev_alloc((void **)&h->d_gw, sizeof(double) * NG)) {
        rt_destroy(h);
        return RT_ENOMEM;
    }
    std::vector<double> gw(NG, 1.0);
    if (NG > 1) gw.assign(cfg->gauss_weights, cfg->gauss_weights + NG);
    if (hipMemcpy(h->d_c2lam, c2.data(), sizeof(double) * (NB + 1), hipMemcpyHostToDevice) ||
        hipMemcpy(h->d_c2lam_f, c2f.data(), sizeof(float) * (NB + 1), hipMemcpyHostToDevice) ||
        hipMemcpy(h->d_fstar, cfg->stellar_flux, sizeof(double) * NB, hipMemcpyHostToDevice) ||
        hipMemcpy(h->d_gw, gw.data(), sizeof(double) * NG, hipMemcpyHostToDevice)) {
        rt_destroy(h);
        return RT_EDEVICE;
    }
    *out = h;
    return RT_OK;
}

extern "C" rt_status rt_destroy(rt_handle *h)
{
    if (!h) return RT_OK;
    (void)hipSetDevice(h->cfg.device);
    if (h->wlaunched) {
        // the worker exits once nothing is left to claim (or after its idle bound)
        __atomic_store_n(&h->wq->stop, 1u, __ATOMIC_RELEASE);
        (void)hipEventSynchronize(h->wevent);
    }
    if (h->wevent) (void)hipEventDestroy(h->wevent);
    if (h->wstream) (void)hipStreamDestroy(h->wstream);
    if (h->wq) (void)hipHostFree(h->wq);
    if (h->wring) (void)hipHostFree(h->wring);
    if (h->wslots) (void)hipHostFree(h->wslots);
    if (h->wdone) (void)hipHostFree(h->wdone);
    (void)hipFree(h->d_targs);
    (void)hipFree(h->d_head);
    (void)hipFree(h->d_exiting);
    (void)hipFree(h->d_wgst);
    for (auto &s : h->streams)
        if (s) (void)hipStreamSynchronize(s);
    (void)hipDeviceSynchronize();
    for (auto &b : h->slots) {
        if (b.done) (void)hipEventDestroy(b.done);
        if (b.h_args) (void)hipHostFree(b.h_args);
        if (b.h_first) (void)hipHostFree(b.h_first);
        if (b.h_status) (void)hipHostFree(b.h_status);
        (void)hipFree(b.d_args);
        (void)hipFree(b.d_first);
        (void)hipFree(b.d_status);
    }
    for (auto &s : h->streams)
        if (s) (void)hipStreamDestroy(s);
    (void)hipFree(h->d_c2lam);
    (void)hipFree(h->d_c2lam_f);
    (void)hipFree(h->d_fstar);
    (void)hipFree(h->d_gw);
    (void)hipFree(h->d_opac);
    (void)hipFree(h->d_scratch);
    (void)hipFree(h->arena_mem);
    delete h;
    return RT_OK;
}

// Slabs of a request: one per layer, two on the sub-layer grid.
static int request_slabs(const rt_request *r) { return r->T_center ? 2 * r->n_layers : r->n_layers; }

static rtk::Geometry request_geometry(const rt_handle *h, const rt_request *r)
{
    const int N = request_slabs(r);
    if (r->kernel == RT_KERNEL_DEEP ||
        (r->kernel == RT_KERNEL_AUTO && r->cols_per_block == 0 && prefer_deep(h, r->n_cols, N)))
        return rtk::deep_geometry(r->n_cols, N, h->NBG, h->dev);
    const int kernel = r->kernel == RT_KERNEL_LANE ? rtk::KERNEL_LANE : rtk::KERNEL_LAYER;
    return rtk::solve_geometry(r->n_cols, N, h->NBG, r->cols_per_block, kernel, r->precision,
                               h->dev, h->NG);
}

static rt_status validate(rt_handle *h, const rt_request *r)
{
    if (!r) return fail(h, RT_EINVAL, "request is NULL");
    if (r->n_cols < 1) return fail(h, RT_EINVAL, "n_cols must be >= 1 (got %d)", r->n_cols);
    if (r->n_layers < 1 || r->n_layers > kMaxLayers)
        return fail(h, RT_EINVAL, "n_layers must be in [1, %d] (got %d)", kMaxLayers, r->n_layers);
    if (r->precision != RT_FP64 && r->precision != RT_MIXED)
        return fail(h, RT_EINVAL, "precision must be RT_FP64 or RT_MIXED");
    if (r->kernel < RT_KERNEL_AUTO || r->kernel > RT_KERNEL_DEEP)
        return fail(h, RT_EINVAL, "kernel must be RT_KERNEL_AUTO, _LANE, _LAYER or _DEEP");
    if (r->kernel == RT_KERNEL_DEEP && r->cols_per_block != 0)
        return fail(h, RT_EINVAL, "the deep kernel takes no tile (cols_per_block must be 0)");
    if (r->input_dtype != RT_F64 && r->input_dtype != RT_F32)
        return fail(h, RT_EINVAL, "input_dtype must be RT_F64 or RT_F32");
    if (r->input_dtype == RT_F32 && r->precision != RT_MIXED)
        return fail(h, RT_EINVAL, "FP32 input storage needs the mixed precision (RT_MIXED)");
    if (h->NG > 1 && r->kernel == RT_KERNEL_LANE)
        return fail(h, RT_EINVAL, "Gaussian points per bin need the layer kernel");
    if (r->cols_per_block < 0) return fail(h, RT_EINVAL, "cols_per_block must be >= 0");
    if (request_geometry(h, r).threads == 0)
        return fail(h, RT_EINVAL, "tile of %d columns x %d bins does not fit the %s kernel",
                    r->cols_per_block, h->NBG, r->kernel == RT_KERNEL_LANE ? "lane" : "layer");
    const void *req_in[] = {r->p_iface, r->T_iface, r->dtau, r->w0, r->g0, r->mu_star, r->T_int};
    const char *names_in[] = {"p_iface", "T_iface", "dtau", "w0", "g0", "mu_star", "T_int"};
    for (int k = 0; k < 7; ++k)
        if (!req_in[k]) return fail(h, RT_EINVAL, "%s is NULL", names_in[k]);
    const void *req_out[] = {r->F_up, r->F_dn, r->F_beam, r->F_net, r->heating};
    const char *names_out[] = {"F_up", "F_dn", "F_beam", "F_net", "heating"};
    for (int k = 0; k < 5; ++k)
        if (!req_out[k]) return fail(h, RT_EINVAL, "%s is NULL", names_out[k]);
    if (r->T_center) {
        if (r->kernel == RT_KERNEL_LANE)
            return fail(h, RT_EINVAL, "the sub-layer grid needs the layer kernel");
        if (!r->p_center) return fail(h, RT_EINVAL, "p_center is NULL (T_center is set)");
        if (!r->F_up_center || !r->F_dn_center || !r->F_beam_center || !r->F_net_center)
            return fail(h, RT_EINVAL, "the sub-layer grid needs all four centre outputs");
        if (2 * r->n_layers > kMaxLayers)
            return fail(h, RT_EINVAL, "2 x n_layers must be <= %d", kMaxLayers);
    } else if (r->p_center || r->F_up_center || r->F_dn_center || r->F_beam_center ||
               r->F_net_center) {
        return fail(h, RT_EINVAL, "centre arrays given without T_center");
    }
    const void *all[] = {r->p_iface, r->T_iface, r->dtau, r->w0, r->g0, r->mu_star, r->T_int,
                         r->F_toa, r->F_up, r->F_dn, r->F_beam, r->F_net, r->heating, r->dTdt,
                         r->F_up_toa_bin, r->F_up_bin, r->F_dn_bin, r->flags, r->T_center,
                         r->p_center, r->F_up_center, r->F_dn_center, r->F_beam_center,
                         r->F_net_center};
    for (const void *p : all)
        if (p && (reinterpret_cast<uintptr_t>(p) % (p == r->flags ? 4 : 8)))
            return fail(h, RT_EINVAL, "misaligned pointer %p", p);
    const long long lanes = (long long)r->n_cols * h->NBG;
    if (lanes * (request_slabs(r) + 1) > (1ll << 40))
        return fail(h, RT_EINVAL, "problem too large");
    return RT_OK;
}

static rtk::SolveArgs make_args(const rt_handle *h, const rt_request *r, double *scratch)
{
    rtk::SolveArgs a{};
    a.C = r->n_cols;
    a.N = request_slabs(r);
    a.sub = r->T_center ? 1 : 0;
    a.Tc = r->T_center;
    a.pc = r->p_center;
    a.F_up_c = r->F_up_center;
    a.F_dn_c = r->F_dn_center;
    a.F_beam_c = r->F_beam_center;
    a.F_net_c = r->F_net_center;
    a.NB = h->NBG;
    a.NG = h->NG;
    a.wg = h->d_gw;
    a.c2_over_lam = h->d_c2lam;
    a.c2_over_lam_f = h->d_c2lam_f;
    a.F_star = h->d_fstar;
    a.p = r->p_iface;
    a.T = r->T_iface;
    a.dtau = static_cast<const double *>(r->dtau);
    a.w0 = static_cast<const double *>(r->w0);
    a.g0 = static_cast<const double *>(r->g0);
    a.in_f32 = r->input_dtype == RT_F32;
    a.mu = r->mu_star;
    a.Tint = r->T_int;
    a.Ftoa = r->F_toa;
    a.F_up = r->F_up;
    a.F_dn = r->F_dn;
    a.F_beam = r->F_beam;
    a.F_net = r->F_net;
    a.heat = r->heating;
    a.dTdt = r->dTdt;
    a.F_up_toa_bin = r->F_up_toa_bin;
    a.F_up_bin = r->F_up_bin;
    a.F_dn_bin = r->F_dn_bin;
    a.flags = r->flags;
    a.scratch = scratch;
    a.o.improved = h->cfg.improved;
    a.o.noniso = h->cfg.noniso;
    a.o.e_clamp = h->cfg.e_clamp;
    a.o.eps2 = h->cfg.eps2;
    a.o.e_tau = h->cfg.e_tau;
    a.o.g_guard = h->cfg.g_guard;
    a.o.gravity = h->cfg.gravity;
    a.o.cp = h->cfg.cp;
    return a;
}

extern "C" rt_status rt_set_opacities(rt_handle *h, const rt_opacities *op)
{
    if (!h || !op) return RT_EINVAL;
    const int nT = op->n_temp, nP = op->n_press, NB = h->NB, NBG = h->NBG;
    if (nT < 2 || nT > 1024 || nP < 2 || nP > 1024 || !op->temp || !op->log10p || !op->kappa)
        return fail(h, RT_EINVAL, "table grid must be 2..1024 x 2..1024 with all arrays given");
    for (int i = 0; i < nT; ++i)
        if (!std::isfinite(op->temp[i]) || (i > 0 && !(op->temp[i] > op->temp[i - 1])))
            return fail(h, RT_EINVAL, "temperature grid must be finite and strictly ascending");
    for (int j = 0; j < nP; ++j)
        if (!std::isfinite(op->log10p[j]) || (j > 0 && !(op->log10p[j] > op->log10p[j - 1])))
            return fail(h, RT_EINVAL, "log10 pressure grid must be finite and strictly ascending");
    const size_t nk = (size_t)nP * nT * NBG;
    for (size_t k = 0; k < nk; ++k)
        if (!(op->kappa[k] >= 0.0) || !std::isfinite(op->kappa[k]))
            return fail(h, RT_EINVAL, "kappa must be finite and >= 0");
    const bool cloud = op->cloud_abs != nullptr;
    if (cloud != (op->cloud_scat != nullptr) || cloud != (op->cloud_g0 != nullptr))
        return fail(h, RT_EINVAL, "condensate arrays: all three or none");
    if (!(op->m_mean > 0.0) || !(op->f_cloud >= 0.0) || !(op->x_h2 >= 0.0) || !(op->x_he >= 0.0) ||
        !std::isfinite(op->f_cloud) || !std::isfinite(op->x_h2) || !std::isfinite(op->x_he))
        return fail(h, RT_EINVAL, "m_mean > 0; f_cloud, x_h2, x_he finite and >= 0");
    std::vector<double> host(nT + nP + nk + 4 * (size_t)NB);
    std::copy(op->temp, op->temp + nT, host.begin());
    std::copy(op->log10p, op->log10p + nP, host.begin() + nT);
    std::copy(op->kappa, op->kappa + nk, host.begin() + nT + nP);
    double *pb = host.data() + nT + nP + nk;   // per-bin: gas scattering, f abs, f scat, g0
    for (int b = 0; b < NB; ++b) {
        const double lo = h->lam[b], hi = h->lam[b + 1];
        pb[b] = rtk::rayleigh_bin_average(lo, hi, op->x_h2, op->x_he);
        double sa = 0.0, ss = 0.0, g = 0.0;
        if (cloud) {
            sa = op->cloud_abs[b];
            ss = op->cloud_scat[b];
            g = op->cloud_g0[b];
            if (!(sa >= 0.0) || !(ss >= 0.0) || !(g > -1.0 && g < 1.0) || !std::isfinite(sa) ||
                !std::isfinite(ss))
                return fail(h, RT_EINVAL, "condensate cross sections >= 0, asymmetry in (-1, 1)");
        }
        pb[NB + b] = op->f_cloud * sa;
        pb[2 * NB + b] = op->f_cloud * ss;
        pb[3 * NB + b] = g;
    }
    (void)hipSetDevice(h->cfg.device);
    (void)hipDeviceSynchronize();
    (void)hipFree(h->d_opac);
    h->d_opac = nullptr;
    h->have_opac = false;
    if (!dev_alloc((void **)&h->d_opac, host.size() * sizeof(double)))
        return fail(h, RT_ENOMEM, "opacity tables of %zu bytes", host.size() * sizeof(double));
    if (hipMemcpy(h->d_opac, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice) !=
        hipSuccess)
        return fail(h, RT_EDEVICE, "opacity table upload");
    h->opac_nT = nT;
    h->opac_nP = nP;
    h->opac_m = op->m_mean;
    h->have_opac = true;
    return RT_OK;
}

extern "C" rt_status rt_optical_properties(rt_handle *h, const rt_optics_request *r, void *stream)
{
    if (!h) return RT_EINVAL;
    if (!r) return fail(h, RT_EINVAL, "request is NULL");
    if (!h->have_opac) return fail(h, RT_EINVAL, "no opacity tables: call rt_set_opacities");
    if (r->n_cols < 1 || r->n_layers < 1 || r->n_layers > kMaxLayers)
        return fail(h, RT_EINVAL, "n_cols >= 1 and n_layers in [1, %d]", kMaxLayers);
    if ((r->sublayer != 0 && r->sublayer != 1) || r->reserved != 0)
        return fail(h, RT_EINVAL, "sublayer must be 0 or 1, reserved 0");
    const void *ptrs[] = {r->p_iface, r->T_iface, r->p_center, r->T_center, r->dtau, r->w0, r->g0};
    for (const void *p : ptrs) {
        if (!p) return fail(h, RT_EINVAL, "a required array is NULL");
        if (reinterpret_cast<uintptr_t>(p) % 8) return fail(h, RT_EINVAL, "misaligned pointer %p", p);
    }
    (void)hipSetDevice(h->cfg.device);
    rtk::OpticsArgs a{};
    a.C = r->n_cols;
    a.S = r->sublayer ? 2 * r->n_layers : r->n_layers;
    a.NBG = h->NBG;
    a.NG = h->NG;
    a.sub = r->sublayer;
    a.nT = h->opac_nT;
    a.nP = h->opac_nP;
    a.temp = h->d_opac;
    a.log10p = a.temp + a.nT;
    a.kappa = a.log10p + a.nP;
    a.sig_gas = a.kappa + (size_t)a.nP * a.nT * a.NBG;
    a.sig_cl_abs = a.sig_gas + h->NB;
    a.sig_cl_scat = a.sig_cl_abs + h->NB;
    a.g0_cl = a.sig_cl_scat + h->NB;
    a.m_mean = h->opac_m;
    a.gravity = h->cfg.gravity;
    a.p = r->p_iface;
    a.T = r->T_iface;
    a.pc = r->p_center;
    a.Tc = r->T_center;
    a.dtau = r->dtau;
    a.w0 = r->w0;
    a.g0 = r->g0;
    const hipError_t e = rtk::launch_optics(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(h, e, "optics launch");
    return RT_OK;
}

extern "C" rt_status rt_solve_fluxes(rt_handle *h, const rt_request *r, void *stream)
{
    if (!h) return RT_EINVAL;
    rt_status st = validate(h, r);
    if (st != RT_OK) return st;
    (void)hipSetDevice(h->cfg.device);
    const rtk::Geometry g = request_geometry(h, r);
    const size_t need = g.scratch;
    if (need > h->scratch_bytes) {
        // growth waits for the device: earlier solves may still use the old buffer
        (void)hipDeviceSynchronize();
        (void)hipFree(h->d_scratch);
        h->d_scratch = nullptr;
        h->scratch_bytes = 0;
        if (!dev_alloc((void **)&h->d_scratch, need))
            return fail(h, RT_ENOMEM, "work buffer of %zu bytes", need);
        h->scratch_bytes = need;
    }
    rtk::SolveArgs a = make_args(h, r, h->d_scratch);
    hipError_t e = g.kernel == rtk::KERNEL_DEEP
                       ? rtk::launch_deep(a, g, r->precision, (hipStream_t)stream)
                       : rtk::launch_solve(a, g, r->precision, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(h, e, "solve launch");
    return RT_OK;
}

extern "C" rt_status rt_solve_fluxes_noalloc(rt_handle *h, const rt_request *r, void *stream)
{
    if (!h) return RT_EINVAL;
    rt_status st = validate(h, r);
    if (st != RT_OK) return st;
    (void)hipSetDevice(h->cfg.device);
    const rtk::Geometry g = request_geometry(h, r);
    if (g.scratch > kStaticScratchBytes)
        return fail(h, RT_ENOMEM, "request needs a work buffer of %zu bytes; the static one holds %zu",
                    g.scratch, kStaticScratchBytes);
    // the kernels write every word of the work buffer they read later, so it
    // needs no clearing between calls
    rtk::SolveArgs a = make_args(h, r, h->static_ws);
    hipError_t e = g.kernel == rtk::KERNEL_DEEP
                       ? rtk::launch_deep(a, g, r->precision, (hipStream_t)stream)
                       : rtk::launch_solve(a, g, r->precision, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(h, e, "solve launch");
    return RT_OK;
}

extern "C" int32_t rt_request_kernel(rt_handle *h, const rt_request *r)
{
    if (!h) return RT_EINVAL;
    const rt_status st = validate(h, r);
    if (st != RT_OK) return st;
    switch (request_geometry(h, r).kernel) {
    case rtk::KERNEL_LANE: return RT_KERNEL_LANE;
    case rtk::KERNEL_DEEP: return RT_KERNEL_DEEP;
    default: return RT_KERNEL_LAYER;
    }
}

// ---------------------------------------------------------------- serving
static rt_status ensure_serving(rt_handle *h)
{
    if (h->arena_mem) return RT_OK;
    for (auto &s : h->streams)
        if (!s && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
            return fail(h, RT_EDEVICE, "stream creation failed");
    for (int i = 0; i < kSlots; ++i) {
        Batch &b = h->slots[i];
        if (!host_alloc((void **)&b.h_args, sizeof(rtk::SolveArgs) * kMaxBatch) ||
            !host_alloc((void **)&b.h_first, sizeof(int) * kMaxBatch) ||
            !dev_alloc((void **)&b.d_args, sizeof(rtk::SolveArgs) * kMaxBatch) ||
            !dev_alloc((void **)&b.d_first, sizeof(int) * kMaxBatch) ||
            !host_alloc((void **)&b.h_status, sizeof(uint32_t) * kMaxBatch) ||
            !dev_alloc((void **)&b.d_status, sizeof(uint32_t) * kMaxBatch) ||
            hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess)
            return fail(h, RT_ENOMEM, "serving descriptor buffers");
        b.stream = i % kStreams;
    }
    size_t bytes = (size_t)h->cfg.hbm_budget_bytes;
    if (!dev_alloc((void **)&h->arena_mem, bytes)) {
        h->arena_mem = nullptr;
        return fail(h, RT_ENOMEM, "serving arena of %zu bytes", bytes);
    }
    h->arena.reset((char *)h->arena_mem, bytes);
    return RT_OK;
}

// Pinned host memory that the GPU reads and writes coherently; *dev is the
// device's address of it.
template <class T>
static bool host_coherent(T **host, T **dev, size_t n)
{
    void *p = nullptr;
    if (hipHostMalloc(&p, sizeof(T) * n, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    std::memset(p, 0, sizeof(T) * n);
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(p);
        return false;
    }
    *host = static_cast<T *>(p);
    *dev = static_cast<T *>(d);
    return true;
}

// The persistent worker's buffers (once per handle).
static rt_status ensure_worker(rt_handle *h)
{
    if (h->wq) return RT_OK;
    rtk::WorkerArgs &w = h->wargs;
    rtk::WorkQueueHost *q = nullptr, *qd = nullptr;
    rtk::WorkTile *ring = nullptr, *ringd = nullptr;
    rtk::SlotArgs *slots = nullptr, *slotsd = nullptr;
    unsigned int *done = nullptr, *doned = nullptr;
    if (!host_coherent(&q, &qd, 1)) return fail(h, RT_ENOMEM, "worker control words");
    h->wq = q;
    if (!host_coherent(&ring, &ringd, kRingCap)) return fail(h, RT_ENOMEM, "worker tile ring");
    h->wring = ring;
    if (!host_coherent(&slots, &slotsd, kSlotRing)) return fail(h, RT_ENOMEM, "worker request slots");
    h->wslots = slots;
    if (!host_coherent(&done, &doned, kRingCap)) return fail(h, RT_ENOMEM, "worker completion words");
    h->wdone = done;
    if (!dev_alloc((void **)&h->d_targs, sizeof(rtk::SlotArgs) * (size_t)kRingCap) ||
        !dev_alloc((void **)&h->d_head, sizeof(unsigned long long)) ||
        !dev_alloc((void **)&h->d_exiting, sizeof(unsigned int)) ||
        !dev_alloc((void **)&h->d_wgst, sizeof(unsigned int) * (size_t)std::max(h->dev.n_cu, 1)))
        return fail(h, RT_ENOMEM, "worker counters");
    if (hipMemset(h->d_head, 0, sizeof(unsigned long long)) != hipSuccess ||
        hipStreamCreateWithFlags(&h->wstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->wevent, hipEventDisableTiming) != hipSuccess)
        return fail(h, RT_EDEVICE, "worker stream");
    w.q = qd;
    w.ring = ringd;
    w.slots = slotsd;
    w.done = doned;
    w.targs = h->d_targs;
    w.head = h->d_head;
    w.wg_status = h->d_wgst;
    w.exiting = h->d_exiting;
    w.ring_cap = kRingCap;
    w.idle_polls = kIdlePolls;
    w.lds_top = (int)(h->dev.lds - rtk::kWorkerLdsReserve);
    return RT_OK;
}

// Status of a finished request from the condition bits its columns raised:
// strict-mode E <= w0 (RT_EDOMAIN) before out-of-domain inputs (RT_EINVAL).
static rt_status request_status(rt_handle *h, const Job &j, uint32_t bits)
{
    if (bits & RT_FLAG_EDOMAIN)
        return fail(h, RT_EDOMAIN, "ticket %llu: E <= w0 in strict mode (see flags)",
                    (unsigned long long)j.ticket);
    if (bits & RT_FLAG_INVALID)
        return fail(h, RT_EINVAL, "ticket %llu: input values outside their domain (see flags)",
                    (unsigned long long)j.ticket);
    return RT_OK;
}

// Persistent serving: retire requests whose tiles have all completed, admit
// waiting requests (in arrival order, while a slot, ring space and arena memory
// are free: arguments into the slot, tiles into the ring, then the tail
// published), and launch the worker when unclaimed tiles exist and no worker
// is running (it exits after its idle bound).
static void pump_worker(rt_handle *h)
{
    if (!h->wq || h->wbroken) return;
    uint64_t oldest = h->wpublished, oldest_seq = h->wseq;
    for (auto it = h->prunning.begin(); it != h->prunning.end();) {
        PJob &p = it->second;
        while (p.seen < p.ntiles) {
            const unsigned v =
                __atomic_load_n(&h->wdone[(p.first + p.seen) & (kRingCap - 1)], __ATOMIC_ACQUIRE);
            if (!v) break;
            p.bits |= v & 0x7fffffffu;
            ++p.seen;
        }
        if (p.seen == p.ntiles) {
            h->arena.release(p.j.off, p.j.bytes);
            h->finished[p.j.ticket] = request_status(h, p.j, p.bits);
            it = h->prunning.erase(it);
            continue;
        }
        oldest = std::min(oldest, p.first);
        oldest_seq = std::min(oldest_seq, p.seq);
        ++it;
    }
    bool running = false;
    if (h->wlaunched) {
        const hipError_t q = hipEventQuery(h->wevent);
        running = q == hipErrorNotReady;
        if (!running && q != hipSuccess) {
            (void)hipGetLastError();
            hip_fail(h, q, "serving worker");
            for (auto &kv : h->prunning) {
                h->arena.release(kv.second.j.off, kv.second.j.bytes);
                h->finished[kv.first] = RT_EDEVICE;
            }
            h->prunning.clear();
            for (const Job &j : h->pqueued) h->finished[j.ticket] = RT_EDEVICE;
            h->pqueued.clear();
            h->wlaunched = false;
            // published tiles of the failed requests stay in the ring: no
            // later worker may take them
            h->wbroken = true;
            return;
        }
    }
    bool published = false, need_new_life = false;
    while (!h->pqueued.empty()) {
        Job &j = h->pqueued.front();
        const int nt = j.g.blocks;
        if (h->wpublished + nt - oldest > (uint64_t)kRingCap) break;
        // a slot still held by a running request is never reused
        if (h->wseq >= oldest_seq + kSlotRing) break;
        // a slot last used by a request the running worker may have read waits
        // for the next worker lifetime
        if (running && h->wseq >= h->wgen + kSlotRing) {
            need_new_life = true;
            break;
        }
        // likewise a ring position (and its argument copy) the running worker
        // may have claimed
        if (running && h->wpublished + nt > h->wlife0 + kRingCap) {
            need_new_life = true;
            break;
        }
        size_t off;
        if (!h->arena.alloc(j.bytes, &off)) break;   // keep arrival order under pressure
        j.off = off;
        PJob p;
        p.j = j;
        p.seq = h->wseq++;
        p.slot = (int)(p.seq % kSlotRing);
        p.first = h->wpublished;
        p.ntiles = nt;
        rtk::SlotArgs sa{};
        sa.a = make_args(h, &j.req, (double *)(h->arena.base + off));
        sa.a.K = j.g.K;
        sa.a.PC = j.g.PC;
        sa.a.CH = j.g.CH;
        sa.a.L = j.g.lanes;
        sa.mixed = j.req.precision == RT_MIXED;
        h->wslots[p.slot] = sa;
        for (int t = 0; t < nt; ++t) {
            const uint64_t idx = (p.first + t) & (kRingCap - 1);
            h->wdone[idx] = 0u;
            h->wring[idx] = rtk::WorkTile{p.slot, t};
        }
        h->wpublished += nt;
        h->prunning[j.ticket] = p;
        h->pqueued.pop_front();
        published = true;
    }
    if (published) __atomic_store_n(&h->wq->tail, (unsigned long long)h->wpublished, __ATOMIC_RELEASE);
    // ask the running worker to end its lifetime once it has drained its tiles
    __atomic_store_n(&h->wq->stop, need_new_life ? 1u : 0u, __ATOMIC_RELEASE);
    if (running || h->prunning.empty()) return;
    // no worker running: every tile an earlier worker claimed has completed, so
    // the requests still running have unclaimed tiles
    uint64_t gen = h->wseq;
    for (const auto &kv : h->prunning) gen = std::min(gen, kv.second.seq);
    h->wgen = gen;
    h->wlife0 = oldest;
    __atomic_store_n(&h->wq->stop, 0u, __ATOMIC_RELEASE);
    hipError_t e = hipMemsetAsync(h->d_exiting, 0, sizeof(unsigned int), h->wstream);
    if (e == hipSuccess) e = rtk::launch_worker(h->wargs, h->dev, h->wstream);
    if (e == hipSuccess) e = hipEventRecord(h->wevent, h->wstream);
    if (e != hipSuccess) {
        // no worker will take these tiles: fail what was admitted or waits
        (void)hipGetLastError();
        hip_fail(h, e, "serving worker launch");
        for (auto &kv : h->prunning) {
            h->arena.release(kv.second.j.off, kv.second.j.bytes);
            h->finished[kv.first] = RT_EDEVICE;
        }
        h->prunning.clear();
        for (const Job &j : h->pqueued) h->finished[j.ticket] = RT_EDEVICE;
        h->pqueued.clear();
        h->wbroken = true;
        return;
    }
    h->wlaunched = true;
    if (!h->pqueued.empty()) pump_worker(h);   // admit what waited for this lifetime
}

// Retire finished batches, then admit queued requests: in arrival order, by
// device-memory footprint, grouped by (precision, tile) into batched launches.
static void pump(rt_handle *h)
{
    pump_worker(h);
    for (int i = 0; i < kSlots; ++i) {
        Batch &b = h->slots[i];
        if (!b.busy) continue;
        hipError_t q = hipEventQuery(b.done);
        if (q == hipErrorNotReady) continue;
        for (size_t k = 0; k < b.jobs.size(); ++k) {
            const Job &j = b.jobs[k];
            h->arena.release(j.off, j.bytes);
            h->running.erase(j.ticket);
            h->finished[j.ticket] = q != hipSuccess ? RT_EDEVICE : request_status(h, j, b.h_status[k]);
        }
        b.jobs.clear();
        b.busy = false;
    }
    while (!h->queued.empty()) {
        int slot = -1;
        for (int i = 0; i < kSlots; ++i)
            if (!h->slots[i].busy) { slot = i; break; }
        if (slot < 0) return;                       // every batch slot in flight
        Batch &b = h->slots[slot];
        const int prec = h->queued.front().req.precision;
        const int in32 = h->queued.front().req.input_dtype;
        const rtk::Geometry g0 = h->queued.front().g;
        hipStream_t s = h->streams[b.stream];
        if (g0.kernel == rtk::KERNEL_DEEP) {
            // a deep request is a sequence of launches of its own
            Job j = h->queued.front();
            size_t off;
            if (!h->arena.alloc(j.bytes, &off)) return;   // head request waits for memory
            j.off = off;
            h->queued.pop_front();
            rtk::SolveArgs a = make_args(h, &j.req, (double *)(h->arena.base + off));
            a.status = b.d_status;
            hipError_t e = hipMemsetAsync(b.d_status, 0, sizeof(uint32_t), s);
            if (e == hipSuccess) e = rtk::launch_deep(a, j.g, prec, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(b.h_status, b.d_status, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipEventRecord(b.done, s);
            if (e != hipSuccess) {
                hip_fail(h, e, "serving launch");
                h->arena.release(j.off, j.bytes);
                h->finished[j.ticket] = RT_EDEVICE;
                return;
            }
            b.jobs.push_back(j);
            b.busy = true;
            h->running[j.ticket] = slot;
            continue;
        }
        int blocks = 0;
        for (auto it = h->queued.begin(); it != h->queued.end() && (int)b.jobs.size() < kMaxBatch;) {
            // one launch shape per batch: same kernel, precision, input storage, tile,
            // threads and LDS
            if (it->req.precision != prec || it->req.input_dtype != in32 ||
                it->g.kernel != g0.kernel || it->g.K != g0.K ||
                it->g.threads != g0.threads || it->g.lds != g0.lds || it->g.PC != g0.PC ||
                it->g.CH != g0.CH) {
                ++it;
                continue;
            }
            size_t off;
            if (!h->arena.alloc(it->bytes, &off)) break;   // keep arrival order under pressure
            Job j = *it;
            j.off = off;
            rtk::SolveArgs a = make_args(h, &j.req, (double *)(h->arena.base + off));
            a.K = j.g.K;
            a.PC = j.g.PC;
            a.CH = j.g.CH;
            a.L = j.g.lanes;
            a.status = b.d_status + b.jobs.size();
            b.h_args[b.jobs.size()] = a;
            b.h_first[b.jobs.size()] = blocks;
            blocks += j.g.blocks;
            b.jobs.push_back(j);
            it = h->queued.erase(it);
        }
        if (b.jobs.empty()) return;                 // head request waits for memory
        const int n = (int)b.jobs.size();
        hipError_t e = hipMemcpyAsync(b.d_args, b.h_args, sizeof(rtk::SolveArgs) * n,
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b.d_first, b.h_first, sizeof(int) * n, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(b.d_status, 0, sizeof(uint32_t) * n, s);
        if (e == hipSuccess)
            e = rtk::launch_solve_batch(b.d_args, b.d_first, n, blocks, g0, prec, in32, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b.h_status, b.d_status, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(b.done, s);
        if (e != hipSuccess) {
            hip_fail(h, e, "serving launch");
            for (const Job &j : b.jobs) {
                h->arena.release(j.off, j.bytes);
                h->finished[j.ticket] = RT_EDEVICE;
            }
            b.jobs.clear();
            return;
        }
        b.busy = true;
        for (const Job &j : b.jobs) h->running[j.ticket] = slot;
    }
}

extern "C" rt_status rt_submit(rt_handle *h, const rt_request *r, uint64_t *ticket)
{
    if (!h || !ticket) return RT_EINVAL;
    rt_status st = validate(h, r);
    if (st != RT_OK) return st;
    (void)hipSetDevice(h->cfg.device);
    if ((st = ensure_serving(h)) != RT_OK) return st;
    auto inflight = [&] {
        return (int)(h->queued.size() + h->running.size() + h->pqueued.size() + h->prunning.size());
    };
    if (inflight() >= h->cfg.max_inflight) {
        pump(h);
        if (inflight() >= h->cfg.max_inflight)
            return fail(h, RT_EBUSY, "%d requests in flight", h->cfg.max_inflight);
    }
    Job j;
    j.ticket = h->next_ticket++;
    j.req = *r;
    j.g = request_geometry(h, r);
    // the persistent worker takes layer-kernel requests with FP64 input storage;
    // the others (deep and lane kernels, FP32 inputs) run as batched launches
    bool worker = false;
    if (h->cfg.serve_mode == RT_SERVE_PERSISTENT && !h->wbroken && j.g.kernel == rtk::KERNEL_LAYER &&
        r->input_dtype == RT_F64) {
        const rtk::Geometry gw = rtk::worker_geometry(r->n_cols, request_slabs(r), h->NBG, r->precision,
                                                      h->dev, h->NG);
        if (gw.threads > 0 && gw.blocks <= kRingCap) {
            if ((st = ensure_worker(h)) != RT_OK) return st;
            j.g = gw;
            worker = true;
        }
    }
    j.bytes = j.g.scratch;
    if (j.bytes > h->arena.size)
        return fail(h, RT_ENOMEM, "request needs %zu bytes, budget is %zu", j.bytes, h->arena.size);
    (worker ? h->pqueued : h->queued).push_back(j);
    *ticket = j.ticket;
    pump(h);
    return RT_OK;
}

extern "C" rt_status rt_poll(rt_handle *h, uint64_t ticket)
{
    if (!h) return RT_EINVAL;
    (void)hipSetDevice(h->cfg.device);
    pump(h);
    auto f = h->finished.find(ticket);
    if (f != h->finished.end()) {
        rt_status s = f->second;
        h->finished.erase(f);
        return s;
    }
    if (h->running.count(ticket) || h->prunning.count(ticket)) return RT_PENDING;
    for (const Job &j : h->queued)
        if (j.ticket == ticket) return RT_PENDING;
    for (const Job &j : h->pqueued)
        if (j.ticket == ticket) return RT_PENDING;
    return fail(h, RT_ENOTFOUND, "ticket %llu", (unsigned long long)ticket);
}

extern "C" rt_status rt_wait(rt_handle *h, uint64_t ticket)
{
    if (!h) return RT_EINVAL;
    for (;;) {
        rt_status s = rt_poll(h, ticket);
        if (s != RT_PENDING) return s;
        auto it = h->running.find(ticket);
        if (it != h->running.end()) {
            (void)hipEventSynchronize(h->slots[it->second].done);
        } else if (h->prunning.count(ticket) || h->pqueued.size()) {
            // on the persistent worker: completion words in host memory
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        } else {
            // queued behind memory or slots: wait for any batch in flight
            for (auto &b : h->slots)
                if (b.busy) {
                    (void)hipEventSynchronize(b.done);
                    break;
                }
        }
    }
}

// Host side of the libgpweno C ABI (declared in include/gpweno.h).
//
// A context holds the grid, the pre-simulation tables (binary128 -> float64 /
// float32), the options and a small device control block. The caller binds its
// own device state and workspace. A step is a fixed sequence of 3 * ndim sweep
// launches on the context's stream: stage k = 1..3, one sweep per direction.
// Every sweep derives the step's dt (CFL speed of U^n) from the control block;
// the last direction of each stage forms the SSP-RK3 stage output; stage 3
// writes U^{n+1} in place, reduces its CFL speed for the next step, and its
// last block advances t and the step count.
// Because dt, t and the stop condition live on the device, a run replays a
// sequence of captured HIP graph replays and synchronises once per sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/gpweno.h"
#include "gp_tables.h"
#include "gpweno_kernels.h"

namespace {

constexpr int NPART = 1024;         // partial sums of the conservation reduction
// Steps per captured graph. A run of n steps replays them largest first (the
// binary digits of n below 32), so it launches exactly the steps it asks for
// with at most six replays per 63 steps.
constexpr int NGRAPH = 6;
constexpr int GRAPH_STEPS[NGRAPH] = {32, 16, 8, 4, 2, 1};
// Steps enqueued between two reads of the control block in gpweno_run.
constexpr long long RUN_CHUNK = 256;
// A float64 context needs tables accurate to this (gpweno_table_residual).
constexpr double FP64_TABLE_RESIDUAL = 1e-13;

thread_local std::string g_tls_error = "";

// Control blocks (device) and their pinned host mirrors come from a pool per
// device, allocated in chunks and never returned, so that creating and
// destroying contexts (a serving loop admits and retires problems all the
// time) calls no hipMalloc or hipFree, which would synchronise the device.
constexpr int CTL_CHUNK = 64;

struct CtlPool {
    std::vector<gpw::Ctl*> dev, host;
};

std::mutex g_pool_mu;
std::vector<CtlPool> g_pools;

hipError_t ctl_acquire(int device, gpw::Ctl** d, gpw::Ctl** h) {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if ((int)g_pools.size() <= device) g_pools.resize(device + 1);
    CtlPool& p = g_pools[device];
    if (p.dev.empty()) {
        gpw::Ctl *dc = nullptr, *hc = nullptr;
        hipError_t e = hipMalloc(&dc, sizeof(gpw::Ctl) * CTL_CHUNK);
        if (e != hipSuccess) return e;
        e = hipHostMalloc(&hc, sizeof(gpw::Ctl) * CTL_CHUNK, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipFree(dc);
            return e;
        }
        for (int i = CTL_CHUNK - 1; i >= 0; --i) {
            p.dev.push_back(dc + i);
            p.host.push_back(hc + i);
        }
    }
    *d = p.dev.back();
    *h = p.host.back();
    p.dev.pop_back();
    p.host.pop_back();
    return hipSuccess;
}

void ctl_release(int device, gpw::Ctl* d, gpw::Ctl* h) {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (device < 0 || device >= (int)g_pools.size() || !d || !h) return;
    g_pools[device].dev.push_back(d);
    g_pools[device].host.push_back(h);
}

// Scratch of gpweno_step_noalloc, the entry point for callers that cannot
// allocate: the two RK stage states and the direction accumulator of one step,
// in a fixed device array that every GPU the library runs on holds until the
// process ends. Host code reaches it only through the per-device address
// hipGetSymbolAddress returns (taken once per device in gpweno_init_scheme,
// with that device current); the array's name is not a device address on the
// host.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

std::once_flag g_scratch_once[NOALLOC_MAX_DEVICES];
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
hipError_t g_scratch_err[NOALLOC_MAX_DEVICES] = {};

// Once per device, with that device current.
void scratch_setup(int dev) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return;
    std::call_once(g_scratch_once[dev], [dev] {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_err[dev] = e;
        g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
    });
}

}  // namespace

struct gpweno_ctx {
    gpweno_grid grid;
    int R;
    int scheme;                     // gpweno_scheme
    double ell, sigma, gamma;
    double dx[3];
    long long ncell;
    int nv;
    gpweno_options opt;
    GpTablesF64 tab64[3];
    GpAoTablesF64 ao64[3];          // adaptive-order GP only
    gpw::Tab<double> tabd[3];
    gpw::Tab<float> tabf[3];
    double residual = 0.0;          // largest mirror residual of the tables over the axes
    // the step state as last read from the device (t, dt, step count) and
    // whether it is known to hold (set_time makes it exact; a step or batch run
    // outdates it). gpweno_run uses it only to size its first chunk of steps.
    gpw::StepRec shadow{0.0, 0.0, 0, 0};
    bool shadow_ok = false;
    int device;
    gpw::Ctl* d_ctl = nullptr;
    gpw::Ctl* h_ctl = nullptr;      // pinned mirror
    hipStream_t own_stream = nullptr;
    double* state = nullptr;
    double* U1 = nullptr;
    double* U2 = nullptr;
    double* dU = nullptr;
    double* partials = nullptr;
    hipGraphExec_t graph[NGRAPH] = {};  // GRAPH_STEPS[i] steps each
    std::string err;
};

namespace {

int fail(gpweno_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_tls_error = buf;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                         \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail((ctx), GPWENO_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

hipStream_t user_stream(const gpweno_ctx* c) { return static_cast<hipStream_t>(c->opt.stream); }

void drop_graph(gpweno_ctx* c) {
    for (auto& g : c->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

bool has_graph(const gpweno_ctx* c) {
    for (auto g : c->graph)
        if (g) return true;
    return false;
}

// Terms of the flux correction, and the cells a 64-lane run produces with them.
int corr_terms(const gpweno_ctx* c) { return c->opt.flux_corr_terms; }
int run_cells(const gpweno_ctx* c) { return gpw::run_out(corr_terms(c)); }

template <typename Real>
gpw::SweepArgs<Real> base_args(const gpweno_ctx* c, int dir) {
    gpw::SweepArgs<Real> a;
    std::memset(&a, 0, sizeof a);
    for (int d = 0; d < 3; ++d) a.n[d] = d < c->grid.ndim ? c->grid.n[d] : 1;
    a.nseg = (a.n[dir] + run_cells(c) - 1) / run_cells(c);
    a.ncell = c->ncell;
    a.inv_dx = 1.0 / c->dx[dir];
    for (int d = 0; d < 3; ++d) a.inv_dx_all[d] = d < c->grid.ndim ? 1.0 / c->dx[d] : 0.0;
    a.gamma = c->gamma;
    a.inv_gm1 = 1.0 / (c->gamma - 1.0);
    a.positivity = c->opt.positivity_fallback ? 1 : 0;
    a.bc[0] = c->grid.bc[dir][0];
    a.bc[1] = c->grid.bc[dir][1];
    a.ctl = c->d_ctl;
    if constexpr (sizeof(Real) == 8) a.tab = c->tabd[dir];
    else a.tab = c->tabf[dir];
    return a;
}

// Direction of the j-th sweep of an RK stage: z, y, then x. The last sweep
// finishes the stage (RK combination, physical check, CFL speed), and running
// it along x keeps that epilogue's reads and writes contiguous per wave
// without a transpose through LDS.
int sweep_dir(int ndim, int j) { return ndim - 1 - j; }

// Smoothness-indicator kind of the kernels (see launch_sweep).
int indicator_kind(const gpweno_ctx* c) {
    if (c->scheme == GPWENO_GP_AO) return 3;
    if (c->scheme == GPWENO_WENO_JS) return 1;
    return c->opt.nonzero_mean ? 2 : 0;
}

// True when an axis has a non-periodic side (its sweeps need the general
// boundary kernels).
bool general_bc(const gpweno_grid& g, int dir) {
    return g.bc[dir][0] != GPWENO_BC_PERIODIC || g.bc[dir][1] != GPWENO_BC_PERIODIC;
}

// One sweep launch (direction dir) in the configured precision.
int launch(gpweno_ctx* c, int dir, const double* in, const double* un, double* acc, double* out, int stage,
           bool fin, bool first, bool step_start, hipStream_t s) {
    const bool fp32 = c->opt.precision == GPWENO_FP32;
    const gpw::LaunchSel k{dir, c->R, fin, indicator_kind(c), general_bc(c->grid, dir), corr_terms(c), false};
    hipError_t e;
    if (fp32) {
        auto a = base_args<float>(c, dir);
        a.U = in; a.Un = un; a.dU = acc; a.Uout = out;
        a.first = first; a.stage = stage; a.step_start = step_start;
        e = gpw::launch_sweep(c->grid.ndim, true, k, &a, 0, s);
    } else {
        auto a = base_args<double>(c, dir);
        a.U = in; a.Un = un; a.dU = acc; a.Uout = out;
        a.first = first; a.stage = stage; a.step_start = step_start;
        e = gpw::launch_sweep(c->grid.ndim, false, k, &a, 0, s);
    }
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "sweep launch (dir %d): %s", dir, hipGetErrorString(e));
    return GPWENO_OK;
}

// The k-th launch of a step: stage k / ndim + 1, sweep j = k % ndim of the
// stage in the direction sweep_dir(ndim, j).
int launch_step_kernel(gpweno_ctx* c, int k, hipStream_t s) {
    const int ndim = c->grid.ndim;
    const int stage = k / ndim + 1, j = k % ndim, dir = sweep_dir(ndim, j);
    const double* ins[3] = {c->state, c->U1, c->U2};
    double* outs[3] = {c->U1, c->U2, c->state};
    return launch(c, dir, ins[stage - 1], c->state, c->dU, outs[stage - 1], stage, j == ndim - 1, j == 0,
                  k == 0, s);
}

int enqueue_step(gpweno_ctx* c, hipStream_t s) {
    for (int k = 0; k < 3 * c->grid.ndim; ++k) {
        int st = launch_step_kernel(c, k, s);
        if (st) return st;
    }
    return GPWENO_OK;
}

int read_ctl(gpweno_ctx* c, hipStream_t s) {
    HIP_TRY(c, hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(gpw::Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    return GPWENO_OK;
}

int check_err(gpweno_ctx* c) {
    if (c->h_ctl->err)
        return fail(c, GPWENO_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or NaN) at cell %lld",
                    (long long)c->h_ctl->bad_cell);
    return GPWENO_OK;
}

// Captures GRAPH_STEPS[i] steps on the private stream (capture records, it does
// not execute); the graph is launched on the caller's stream.
int ensure_graph(gpweno_ctx* c, int i) {
    if (c->graph[i]) return GPWENO_OK;
    hipStream_t s = c->own_stream;
    HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int st = GPWENO_OK;
    for (int k = 0; k < GRAPH_STEPS[i] && st == GPWENO_OK; ++k) st = enqueue_step(c, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph[i], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->graph[i] = nullptr;
        return fail(c, GPWENO_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return GPWENO_OK;
}

// Enqueues exactly n steps as graph replays, largest graphs first. Every size
// is captured the first time any is needed, so that a later run of another
// length does not capture (a few milliseconds) while it is timed.
int enqueue_graph_steps(gpweno_ctx* c, long long n, hipStream_t s) {
    for (int i = 0; i < NGRAPH; ++i) {
        int st = ensure_graph(c, i);
        if (st) return st;
    }
    for (int i = 0; i < NGRAPH; ++i) {
        const long long reps = n / GRAPH_STEPS[i];
        n -= reps * GRAPH_STEPS[i];
        for (long long r = 0; r < reps; ++r) HIP_TRY(c, hipGraphLaunch(c->graph[i], s));
    }
    return GPWENO_OK;
}

// Ghost cells per side a sweep reads: the stencil radius R, the NC face fluxes
// either side of a face that the correction takes, and the face of the
// difference. A reflecting side mirrors that many distinct interior cells.
int ghost_depth(int R, int nc) { return R + 1 + nc; }

bool valid_options(const gpweno_options* o) {
    return o && (o->precision == GPWENO_FP64 || o->precision == GPWENO_FP32) && o->cfl > 0 &&
           std::isfinite(o->cfl) && o->fixed_dt >= 0 && std::isfinite(o->fixed_dt) &&
           (o->flux_corr_terms == 2 || o->flux_corr_terms == 3);
}

bool valid_scheme(int scheme) {
    return scheme == GPWENO_GP_WENO || scheme == GPWENO_WENO_JS || scheme == GPWENO_WENO_GP || scheme == GPWENO_GP_AO;
}

// The constants of the adaptive-order hybrid (App. A): gamma_HI = gamma_LO = 0.85
// and the CWENO linear weights of Eq. (CWENO-lin).
constexpr double AO_GAMMA_HI = 0.85, AO_GAMMA_LO = 0.85;

// Adaptive-order tables: the GP-R2 sub-stencil weights and K_3(sigma) rows
// (scheme GP-WENO, R = 2) with the CWENO linear weights in place of the
// GP-WENO ones, and the 7- and 5-point tables.
int build_ao(double ell_dx, double sigma_dx, GpTablesF64* t, GpAoTablesF64* ao) {
    int st = gpw_build_tables(GPWENO_GP_WENO, 2, ell_dx, sigma_dx, t);
    if (st) return st;
    const double g[3] = {0.5 * (1 - AO_GAMMA_HI) * (1 - AO_GAMMA_LO), (1 - AO_GAMMA_HI) * AO_GAMMA_LO,
                         0.5 * (1 - AO_GAMMA_HI) * (1 - AO_GAMMA_LO)};
    for (int m = 0; m < 4; ++m) {
        t->gam_plus[m] = t->gam_minus[m] = m < 3 ? g[m] : 0.0;
        for (int j = 0; j < 4; ++j) t->gw_plus[m][j] = t->gam_plus[m] * t->w_plus[m][j];  // unused by GP-AO
    }
    return gpw_build_ao_tables(ell_dx, sigma_dx, ao);
}

template <typename Real>
void fill_ao(gpw::AoTab<Real>& t, const GpAoTablesF64& s) {
    for (int j = 0; j < 7; ++j) {
        t.w7p[j] = (Real)s.w7_plus[j];
        for (int i = 0; i < 7; ++i) t.P7[i][j] = (Real)s.P7[i][j];
    }
    for (int j = 0; j < 5; ++j) {
        t.w5p[j] = (Real)s.w5_plus[j];
        for (int i = 0; i < 5; ++i) t.P5[i][j] = (Real)s.P5[i][j];
    }
    for (int k = 0; k < 3; ++k) t.c[k] = (Real)s.c[k];
    t.ghi = (Real)AO_GAMMA_HI;
}

template <typename Real>
void fill_tab(gpw::Tab<Real>& t, const GpTablesF64& s) {
    for (int m = 0; m < 4; ++m) {
        t.gp[m] = (Real)s.gam_plus[m];
        for (int j = 0; j < 4; ++j) {
            t.wp[m][j] = (Real)s.w_plus[m][j];
            t.gwp[m][j] = (Real)s.gw_plus[m][j];
            for (int i = 0; i < 4; ++i) t.P[m][i][j] = (Real)s.P[m][i][j];
        }
        for (int j = 0; j < 2; ++j) t.Ps[m][j] = (Real)s.Ps[m][j];
    }
}

}  // namespace

extern "C" {

int gpweno_compute_tables(int scheme, int R, double ell_over_dx, double sigma_over_dx, double* w_plus,
                          double* w_minus, double* gam_plus, double* gam_minus, double* P) {
    if (!valid_scheme(scheme)) return fail(nullptr, GPWENO_EINVAL, "unknown scheme %d", scheme);
    if (R < 1 || R > 3) return fail(nullptr, GPWENO_EINVAL, "R must be 1, 2 or 3 (got %d)", R);
    if (scheme == GPWENO_WENO_JS && R > 2) return fail(nullptr, GPWENO_EINVAL, "WENO-JS needs R = 1 or 2");
    if (scheme == GPWENO_GP_AO && R < 2) return fail(nullptr, GPWENO_EINVAL, "GP-AO needs R = 2 or 3");
    if (!(ell_over_dx > 0) || !std::isfinite(ell_over_dx) || !(sigma_over_dx > 0) || !std::isfinite(sigma_over_dx))
        return fail(nullptr, GPWENO_EINVAL, "length scales must be positive and finite");
    GpTablesF64 t;
    GpAoTablesF64 ao;
    int st = scheme == GPWENO_GP_AO ? build_ao(ell_over_dx, sigma_over_dx, &t, &ao)
                                    : gpw_build_tables(scheme, R, ell_over_dx, sigma_over_dx, &t);
    if (st) return fail(nullptr, GPWENO_EINVAL, "table construction failed (%d)", st);
    if (w_plus) std::memcpy(w_plus, t.w_plus, sizeof t.w_plus);
    if (w_minus) std::memcpy(w_minus, t.w_minus, sizeof t.w_minus);
    if (gam_plus) std::memcpy(gam_plus, t.gam_plus, sizeof t.gam_plus);
    if (gam_minus) std::memcpy(gam_minus, t.gam_minus, sizeof t.gam_minus);
    if (P) std::memcpy(P, t.P, sizeof t.P);
    return GPWENO_OK;
}

int gpweno_compute_table_residual(int scheme, int R, double ell_over_dx, double sigma_over_dx, double* residual) {
    if (!residual) return fail(nullptr, GPWENO_EINVAL, "NULL residual");
    if (!valid_scheme(scheme)) return fail(nullptr, GPWENO_EINVAL, "unknown scheme %d", scheme);
    if (R < 1 || R > 3) return fail(nullptr, GPWENO_EINVAL, "R must be 1, 2 or 3 (got %d)", R);
    if (scheme == GPWENO_WENO_JS && R > 2) return fail(nullptr, GPWENO_EINVAL, "WENO-JS needs R = 1 or 2");
    if (scheme == GPWENO_GP_AO && R < 2) return fail(nullptr, GPWENO_EINVAL, "GP-AO needs R = 2 or 3");
    if (!(ell_over_dx > 0) || !std::isfinite(ell_over_dx) || !(sigma_over_dx > 0) || !std::isfinite(sigma_over_dx))
        return fail(nullptr, GPWENO_EINVAL, "length scales must be positive and finite");
    GpTablesF64 t;
    GpAoTablesF64 ao;
    int st = scheme == GPWENO_GP_AO ? build_ao(ell_over_dx, sigma_over_dx, &t, &ao)
                                    : gpw_build_tables(scheme, R, ell_over_dx, sigma_over_dx, &t);
    if (st) return fail(nullptr, GPWENO_EINVAL, "table construction failed (%d)", st);
    *residual = scheme == GPWENO_GP_AO ? std::max(t.mirror_residual, ao.mirror_residual) : t.mirror_residual;
    return GPWENO_OK;
}

int gpweno_compute_ao_tables(double ell_over_dx, double sigma_over_dx, double* w7, double* w5, double* P7,
                             double* P5, double* P3, double* c) {
    if (!(ell_over_dx > 0) || !std::isfinite(ell_over_dx) || !(sigma_over_dx > 0) || !std::isfinite(sigma_over_dx))
        return fail(nullptr, GPWENO_EINVAL, "length scales must be positive and finite");
    GpTablesF64 t;
    GpAoTablesF64 ao;
    int st = build_ao(ell_over_dx, sigma_over_dx, &t, &ao);
    if (st) return fail(nullptr, GPWENO_EINVAL, "table construction failed (%d)", st);
    if (w7) {
        std::memcpy(w7, ao.w7_plus, sizeof ao.w7_plus);
        std::memcpy(w7 + 7, ao.w7_minus, sizeof ao.w7_minus);
    }
    if (w5) {
        std::memcpy(w5, ao.w5_plus, sizeof ao.w5_plus);
        std::memcpy(w5 + 5, ao.w5_minus, sizeof ao.w5_minus);
    }
    if (P7) std::memcpy(P7, ao.P7, sizeof ao.P7);
    if (P5) std::memcpy(P5, ao.P5, sizeof ao.P5);
    if (P3) std::memcpy(P3, ao.P3, sizeof ao.P3);
    if (c) std::memcpy(c, ao.c, sizeof ao.c);
    return GPWENO_OK;
}

int gpweno_init(const gpweno_grid* grid, int R, double ell, double sigma, double gamma, gpweno_ctx** out) {
    return gpweno_init_scheme(grid, GPWENO_GP_WENO, R, ell, sigma, gamma, out);
}

int gpweno_init_scheme(const gpweno_grid* grid, int scheme, int R, double ell, double sigma, double gamma,
                       gpweno_ctx** out) {
    if (!grid || !out) return fail(nullptr, GPWENO_EINVAL, "NULL grid or output pointer");
    *out = nullptr;
    if (grid->ndim < 1 || grid->ndim > 3) return fail(nullptr, GPWENO_EINVAL, "ndim must be 1, 2 or 3");
    if (!valid_scheme(scheme)) return fail(nullptr, GPWENO_EINVAL, "unknown scheme %d", scheme);
    if (R < 1 || R > 3) return fail(nullptr, GPWENO_EINVAL, "R must be 1, 2 or 3 (got %d)", R);
    if (scheme == GPWENO_WENO_JS && R > 2) return fail(nullptr, GPWENO_EINVAL, "WENO-JS needs R = 1 or 2");
    if (scheme == GPWENO_GP_AO && R < 2) return fail(nullptr, GPWENO_EINVAL, "GP-AO needs R = 2 or 3");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) return fail(nullptr, GPWENO_EINVAL, "gamma must be > 1");
    if (!(ell > 0) || !std::isfinite(ell)) return fail(nullptr, GPWENO_EINVAL, "ell must be positive");
    gpweno_ctx* c = new (std::nothrow) gpweno_ctx();
    if (!c) return fail(nullptr, GPWENO_ENOMEM, "out of host memory");
    c->grid = *grid;
    c->R = R;
    c->scheme = scheme;
    c->ell = ell;
    c->sigma = sigma;
    c->gamma = gamma;
    c->nv = 2 + grid->ndim;
    c->ncell = 1;
    for (int d = 0; d < 3; ++d) {
        if (d >= grid->ndim) {
            c->grid.n[d] = 1;
            c->grid.bc[d][0] = c->grid.bc[d][1] = GPWENO_BC_PERIODIC;
            c->dx[d] = 1.0;
            continue;
        }
        const int blo = grid->bc[d][0], bhi = grid->bc[d][1];
        if (blo < GPWENO_BC_PERIODIC || blo > GPWENO_BC_REFLECT || bhi < GPWENO_BC_PERIODIC ||
            bhi > GPWENO_BC_REFLECT || ((blo == GPWENO_BC_PERIODIC) != (bhi == GPWENO_BC_PERIODIC))) {
            delete c;
            return fail(nullptr, GPWENO_EINVAL, "axis %d: invalid boundary kinds (%d, %d)", d, blo, bhi);
        }
        if ((blo == GPWENO_BC_REFLECT || bhi == GPWENO_BC_REFLECT) && grid->n[d] < R + 3) {
            delete c;
            return fail(nullptr, GPWENO_EINVAL, "axis %d: a reflecting side needs n >= R + 3", d);
        }
        if (grid->n[d] < 2 || grid->n[d] > (1 << 24)) {
            delete c;
            return fail(nullptr, GPWENO_EINVAL, "axis %d: need 2 <= n <= 2^24 (got %d)", d, grid->n[d]);
        }
        const double len = grid->hi[d] - grid->lo[d];
        if (!(len > 0) || !std::isfinite(len)) {
            delete c;
            return fail(nullptr, GPWENO_EINVAL, "axis %d: hi must exceed lo", d);
        }
        c->dx[d] = len / grid->n[d];
        c->ncell *= grid->n[d];
        if (!(sigma > c->dx[d])) {
            delete c;
            return fail(nullptr, GPWENO_EINVAL, "sigma must exceed dx on every axis (sigma <= dx is unstable)");
        }
        int st = scheme == GPWENO_GP_AO ? build_ao(ell / c->dx[d], sigma / c->dx[d], &c->tab64[d], &c->ao64[d])
                                        : gpw_build_tables(scheme, R, ell / c->dx[d], sigma / c->dx[d], &c->tab64[d]);
        if (st) {
            delete c;
            return fail(nullptr, GPWENO_EINVAL, "table construction failed on axis %d (%d)", d, st);
        }
        fill_tab(c->tabd[d], c->tab64[d]);
        fill_tab(c->tabf[d], c->tab64[d]);
        c->residual = std::max(c->residual, c->tab64[d].mirror_residual);
        if (scheme == GPWENO_GP_AO) {
            fill_ao(c->tabd[d].ao, c->ao64[d]);
            fill_ao(c->tabf[d].ao, c->ao64[d]);
            c->residual = std::max(c->residual, c->ao64[d].mirror_residual);
        }
    }
    if (c->ncell > (1ll << 40)) {
        delete c;
        return fail(nullptr, GPWENO_EINVAL, "grid too large");
    }
    // tables too badly conditioned for float64 parity run in float32 only
    c->opt.precision = c->residual > FP64_TABLE_RESIDUAL ? GPWENO_FP32 : GPWENO_FP64;
    c->opt.cfl = 0.4;
    c->opt.fixed_dt = 0.0;
    c->opt.positivity_fallback = 0;
    c->opt.stream = nullptr;
    c->opt.nonzero_mean = 0;
    c->opt.flux_corr_terms = 2;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) scratch_setup(c->device);
    if (e == hipSuccess) e = ctl_acquire(c->device, &c->d_ctl, &c->h_ctl);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemsetAsync(c->d_ctl, 0, sizeof(gpw::Ctl), c->own_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->own_stream);
    if (e != hipSuccess) {
        int code = fail(nullptr, GPWENO_EHIP, "device set-up: %s", hipGetErrorString(e));
        gpweno_destroy(c);
        return code;
    }
    std::memset(c->h_ctl, 0, sizeof(gpw::Ctl));
    *out = c;
    return GPWENO_OK;
}

int gpweno_set_options(gpweno_ctx* c, const gpweno_options* o) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!valid_options(o)) return fail(c, GPWENO_EINVAL, "invalid options");
    if (o->precision == GPWENO_FP64 && c->residual > FP64_TABLE_RESIDUAL)
        return fail(c, GPWENO_EINVAL,
                    "the tables hold only %.1e relative accuracy (ell/dx too large for R = %d): GPWENO_FP32 only",
                    c->residual, c->R);
    if (o->flux_corr_terms == 3) {
        const bool gp_zero_mean = (c->scheme == GPWENO_GP_WENO || c->scheme == GPWENO_WENO_GP) && !o->nonzero_mean;
        if (!gp_zero_mean)
            return fail(c, GPWENO_EINVAL, "flux_corr_terms = 3 needs GP-WENO or WENO-GP with zero-mean indicators");
    }
    for (int d = 0; d < c->grid.ndim; ++d)
        if ((c->grid.bc[d][0] == GPWENO_BC_REFLECT || c->grid.bc[d][1] == GPWENO_BC_REFLECT) &&
            c->grid.n[d] < ghost_depth(c->R, o->flux_corr_terms))
            return fail(c, GPWENO_EINVAL, "axis %d: a reflecting side needs n >= %d", d,
                        ghost_depth(c->R, o->flux_corr_terms));
    const bool changes_graph = o->precision != c->opt.precision ||
                               o->positivity_fallback != c->opt.positivity_fallback || o->stream != c->opt.stream ||
                               (o->nonzero_mean != 0) != (c->opt.nonzero_mean != 0) ||
                               o->flux_corr_terms != c->opt.flux_corr_terms;
    const bool changes_rule = o->cfl != c->opt.cfl || o->fixed_dt != c->opt.fixed_dt;
    if (changes_graph) {
        // launches of the graphs, or other work on the bound state, may still be
        // in flight on the current stream, and work on a new stream must come
        // after them (a context with neither has nothing to wait for)
        if (c->state || has_graph(c)) HIP_TRY(c, hipStreamSynchronize(user_stream(c)));
        drop_graph(c);
    }
    c->opt = *o;
    if (changes_rule && c->state) {
        // the CFL number and fixed dt live in the control block
        if (read_ctl(c, user_stream(c))) return GPWENO_EHIP;
        hipError_t e = gpw::launch_set_time(c->d_ctl, gpw::current_rec(*c->h_ctl).t,
                                            gpw::current_rec(*c->h_ctl).nsteps, c->opt.cfl, c->opt.fixed_dt,
                                            user_stream(c));
        if (e != hipSuccess) return fail(c, GPWENO_EHIP, "set_time launch: %s", hipGetErrorString(e));
        const double ix[3] = {1.0 / c->dx[0], c->grid.ndim > 1 ? 1.0 / c->dx[1] : 0.0,
                              c->grid.ndim > 2 ? 1.0 / c->dx[2] : 0.0};
        e = gpw::launch_speed(c->grid.ndim, c->state, c->ncell, ix, c->gamma, c->d_ctl, user_stream(c));
        if (e != hipSuccess) return fail(c, GPWENO_EHIP, "speed launch: %s", hipGetErrorString(e));
    }
    return GPWENO_OK;
}

int gpweno_get_options(const gpweno_ctx* c, gpweno_options* o) {
    if (!c || !o) return fail(nullptr, GPWENO_EINVAL, "NULL argument");
    *o = c->opt;
    return GPWENO_OK;
}

size_t gpweno_state_count(const gpweno_ctx* c) { return c ? (size_t)c->nv * (size_t)c->ncell : 0; }

size_t gpweno_workspace_bytes(const gpweno_ctx* c) {
    if (!c) return 0;
    const size_t st = align256(sizeof(double) * (size_t)c->nv * (size_t)c->ncell);
    return 2 * st + (c->grid.ndim > 1 ? st : 0) + align256(sizeof(double) * (size_t)c->nv * NPART);
}

int gpweno_set_time(gpweno_ctx* c, double t, long nsteps) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!c->state) return fail(c, GPWENO_ESTATE, "no state bound");
    if (!std::isfinite(t) || nsteps < 0) return fail(c, GPWENO_EINVAL, "invalid time or step count");
    hipStream_t s = user_stream(c);
    hipError_t e = gpw::launch_set_time(c->d_ctl, t, nsteps, c->opt.cfl, c->opt.fixed_dt, s);
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "set_time launch: %s", hipGetErrorString(e));
    c->shadow = gpw::StepRec{t, 0.0, (long long)nsteps, 0};
    c->shadow_ok = true;
    const double ix[3] = {1.0 / c->dx[0], c->grid.ndim > 1 ? 1.0 / c->dx[1] : 0.0,
                          c->grid.ndim > 2 ? 1.0 / c->dx[2] : 0.0};
    e = gpw::launch_speed(c->grid.ndim, c->state, c->ncell, ix, c->gamma, c->d_ctl, s);
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "speed launch: %s", hipGetErrorString(e));
    return GPWENO_OK;
}

int gpweno_bind(gpweno_ctx* c, double* d_state, void* d_workspace) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!d_state || !d_workspace) return fail(c, GPWENO_EINVAL, "NULL state or workspace");
    if (((uintptr_t)d_state & 7) || ((uintptr_t)d_workspace & 255))
        return fail(c, GPWENO_EINVAL, "state must be 8-byte and workspace 256-byte aligned");
    // the graphs (which hold the old buffers' addresses) may still be running
    if (has_graph(c)) HIP_TRY(c, hipStreamSynchronize(user_stream(c)));
    drop_graph(c);
    const size_t st = align256(sizeof(double) * (size_t)c->nv * (size_t)c->ncell);
    char* w = static_cast<char*>(d_workspace);
    c->state = d_state;
    c->U1 = reinterpret_cast<double*>(w);
    c->U2 = reinterpret_cast<double*>(w + st);
    size_t off = 2 * st;
    if (c->grid.ndim > 1) {
        c->dU = reinterpret_cast<double*>(w + off);
        off += st;
    } else {
        c->dU = nullptr;
    }
    c->partials = reinterpret_cast<double*>(w + off);
    return gpweno_set_time(c, 0.0, 0);
}

int gpweno_step(gpweno_ctx* c, double t_final, double* dt_out) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!c->state) return fail(c, GPWENO_ESTATE, "no state bound");
    hipStream_t s = user_stream(c);
    long long before = 0;
    int st;
    if (dt_out) {
        *dt_out = 0.0;
        if ((st = read_ctl(c, s))) return st;
        before = gpw::current_rec(*c->h_ctl).nsteps;
    }
    hipError_t e = gpw::launch_set_run(c->d_ctl, t_final, LLONG_MAX, s);
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "set_run launch: %s", hipGetErrorString(e));
    c->shadow_ok = false;
    if ((st = enqueue_step(c, s))) return st;
    if (!dt_out) return GPWENO_OK;
    if ((st = read_ctl(c, s))) return st;
    const gpw::StepRec& r = gpw::current_rec(*c->h_ctl);
    if (r.nsteps > before) *dt_out = r.dt;
    return check_err(c);
}

int gpweno_run(gpweno_ctx* c, double t_final, long max_steps, long* nsteps_out, double* t_out) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!c->state) return fail(c, GPWENO_ESTATE, "no state bound");
    if (nsteps_out) *nsteps_out = 0;
    hipStream_t s = user_stream(c);
    // the limit counts from the step count the device holds when the run starts
    hipError_t e = gpw::launch_set_run_rel(c->d_ctl, t_final, max_steps < 0 ? -1 : (long long)max_steps, s);
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "set_run launch: %s", hipGetErrorString(e));
    // steps per chunk: what remains of the step limit, and no more than the last
    // known dt says remain to t_final, so that hardly any enqueued step finds the
    // run already over; one read of the control block per chunk
    long long remaining = max_steps < 0 ? LLONG_MAX : (long long)max_steps;
    gpw::StepRec last = c->shadow;
    bool known = c->shadow_ok;
    double t_prev = 0.0;
    long long n_prev = 0;
    bool first = true;
    int st = GPWENO_OK;
    for (;;) {
        long long plan = std::min(remaining, RUN_CHUNK);
        if (known && last.dt > 0) {
            const double est = (t_final - last.t) / last.dt;
            if (est < (double)plan) plan = std::max(1ll, (long long)est);
        }
        if ((st = enqueue_graph_steps(c, plan, s))) return st;
        if ((st = read_ctl(c, s))) return st;
        const gpw::Ctl& h = *c->h_ctl;
        last = gpw::current_rec(h);
        known = true;
        c->shadow = last;
        c->shadow_ok = true;
        if ((st = check_err(c))) break;
        if (!(last.t < t_final) || last.nsteps >= h.step_limit) break;
        // a chunk that moves neither the step count nor the time cannot finish
        const double t_before = first ? h.run_t0 : t_prev;
        const long long n_before = first ? h.run_start : n_prev;
        if (last.nsteps == n_before || !(last.t > t_before)) {
            st = fail(c, GPWENO_ESTATE, "run stalled at step %lld, t = %.17g (time step %.3g)", last.nsteps, last.t,
                      last.dt);
            break;
        }
        remaining = h.step_limit - last.nsteps;
        t_prev = last.t;
        n_prev = last.nsteps;
        first = false;
    }
    if (nsteps_out) *nsteps_out = (long)(last.nsteps - c->h_ctl->run_start);
    if (t_out) *t_out = last.t;
    return st;
}

int gpweno_get_time(gpweno_ctx* c, double* t, double* dt, long* nsteps) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    int st = read_ctl(c, user_stream(c));
    if (st) return st;
    const gpw::StepRec& r = gpw::current_rec(*c->h_ctl);
    if (t) *t = r.t;
    if (dt) *dt = r.dt;
    if (nsteps) *nsteps = (long)r.nsteps;
    return check_err(c);
}

int gpweno_rhs(gpweno_ctx* c, const double* d_U, double* d_L) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!d_U || !d_L) return fail(c, GPWENO_EINVAL, "NULL state or output");
    const size_t bytes = sizeof(double) * (size_t)c->nv * (size_t)c->ncell;
    const char *u = reinterpret_cast<const char*>(d_U), *l = reinterpret_cast<const char*>(d_L);
    if (u < l + bytes && l < u + bytes) return fail(c, GPWENO_EINVAL, "input and output overlap");
    for (int dir = 0; dir < c->grid.ndim; ++dir) {
        int st = launch(c, dir, d_U, d_U, d_L, d_L, 0, false, dir == 0, false, user_stream(c));
        if (st) return st;
    }
    return GPWENO_OK;
}

int gpweno_rhs_dir(gpweno_ctx* c, int dir, const double* d_U, double* d_L, int accumulate) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!d_U || !d_L) return fail(c, GPWENO_EINVAL, "NULL state or output");
    if (dir < 0 || dir >= c->grid.ndim) return fail(c, GPWENO_EINVAL, "dir must be in [0, ndim)");
    const size_t bytes = sizeof(double) * (size_t)c->nv * (size_t)c->ncell;
    const char *u = reinterpret_cast<const char*>(d_U), *l = reinterpret_cast<const char*>(d_L);
    if (u < l + bytes && l < u + bytes) return fail(c, GPWENO_EINVAL, "input and output overlap");
    return launch(c, dir, d_U, d_U, d_L, d_L, 0, false, accumulate == 0, false, user_stream(c));
}

int gpweno_step_kernel(gpweno_ctx* c, int k) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!c->state) return fail(c, GPWENO_ESTATE, "no state bound");
    if (k < 0 || k >= 3 * c->grid.ndim) return fail(c, GPWENO_EINVAL, "k must be in [0, 3 ndim)");
    c->shadow_ok = false;
    return launch_step_kernel(c, k, user_stream(c));
}

int gpweno_conserved_sums(gpweno_ctx* c, double* out) {
    if (!c || !out) return fail(c, GPWENO_EINVAL, "NULL argument");
    if (!c->state) return fail(c, GPWENO_ESTATE, "no state bound");
    hipStream_t s = user_stream(c);
    hipError_t e = gpw::launch_sums(c->nv, c->state, c->ncell, c->partials, NPART, c->d_ctl, s);
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "sums launch: %s", hipGetErrorString(e));
    int st = read_ctl(c, s);
    if (st) return st;
    for (int k = 0; k < c->nv; ++k) out[k] = c->h_ctl->sums[k];
    return GPWENO_OK;
}

int gpweno_step_noalloc(gpweno_ctx* c, double* d_state, double t_final) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!d_state || ((uintptr_t)d_state & 7)) return fail(c, GPWENO_EINVAL, "state must be non-NULL and 8-byte aligned");
    const size_t st = align256(sizeof(double) * (size_t)c->nv * (size_t)c->ncell);
    const size_t need = 2 * st + (c->grid.ndim > 1 ? st : 0);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(c, GPWENO_EINVAL, "this grid needs %zu bytes of step scratch; the library holds %zu per device",
                    need, NOALLOC_SCRATCH_BYTES);
    if (c->device < 0 || c->device >= NOALLOC_MAX_DEVICES || !g_scratch_ptr[c->device])
        return fail(c, GPWENO_EHIP, "step scratch address of device %d unavailable: %s", c->device,
                    c->device >= 0 && c->device < NOALLOC_MAX_DEVICES ? hipGetErrorString(g_scratch_err[c->device])
                                                                      : "device index out of range");
    char* w = static_cast<char*>(g_scratch_ptr[c->device]);
    double* U1 = reinterpret_cast<double*>(w);
    double* U2 = reinterpret_cast<double*>(w + st);
    double* dU = c->grid.ndim > 1 ? reinterpret_cast<double*>(w + 2 * st) : nullptr;
    hipStream_t s = user_stream(c);
    hipError_t e = gpw::launch_step_prep(c->d_ctl, c->opt.cfl, c->opt.fixed_dt, t_final, s);
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "step prep launch: %s", hipGetErrorString(e));
    const double ix[3] = {1.0 / c->dx[0], c->grid.ndim > 1 ? 1.0 / c->dx[1] : 0.0,
                          c->grid.ndim > 2 ? 1.0 / c->dx[2] : 0.0};
    e = gpw::launch_speed(c->grid.ndim, d_state, c->ncell, ix, c->gamma, c->d_ctl, s);
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "speed launch: %s", hipGetErrorString(e));
    c->shadow_ok = false;
    const int ndim = c->grid.ndim;
    const double* ins[3] = {d_state, U1, U2};
    double* outs[3] = {U1, U2, d_state};
    for (int k = 0; k < 3 * ndim; ++k) {
        const int stage = k / ndim + 1, j = k % ndim;
        int st2 = launch(c, sweep_dir(ndim, j), ins[stage - 1], d_state, dU, outs[stage - 1], stage, j == ndim - 1,
                         j == 0, k == 0, s);
        if (st2) return st2;
    }
    return GPWENO_OK;
}

int gpweno_get_failure(gpweno_ctx* c, int* failed, long* bad_cell) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    int st = read_ctl(c, user_stream(c));
    if (st) return st;
    const bool f = c->h_ctl->err != 0;
    if (failed) *failed = f ? 1 : 0;
    if (bad_cell) *bad_cell = f ? (long)c->h_ctl->bad_cell : -1;
    return GPWENO_OK;
}

int gpweno_get_tables(const gpweno_ctx* c, int dir, double* w_sub, double* gam, double* P) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    gpweno_ctx* cm = const_cast<gpweno_ctx*>(c);  // the error text only
    if (dir < 0 || dir >= c->grid.ndim) return fail(cm, GPWENO_EINVAL, "dir must be in [0, ndim)");
    if (P && c->scheme == GPWENO_WENO_JS)
        return fail(cm, GPWENO_EINVAL, "WENO-JS indicators differ per sub-stencil: pass P = NULL");
    const GpTablesF64& t = c->tab64[dir];
    const int n = (c->scheme == GPWENO_GP_AO ? 2 : c->R) + 1;  // GP-AO: its 3-point sub-stencils
    for (int m = 0; m < n; ++m) {
        if (gam) {
            gam[m] = t.gam_plus[m];
            gam[n + m] = t.gam_minus[m];
        }
        for (int j = 0; j < n; ++j) {
            if (w_sub) {
                w_sub[m * n + j] = t.w_plus[m][j];
                w_sub[n * n + m * n + j] = t.w_minus[m][j];
            }
            if (P) P[m * n + j] = t.P[0][m][j];
        }
    }
    return GPWENO_OK;
}

int gpweno_table_residual(const gpweno_ctx* c, double* residual) {
    if (!c || !residual) return fail(const_cast<gpweno_ctx*>(c), GPWENO_EINVAL, "NULL argument");
    *residual = c->residual;
    return GPWENO_OK;
}

int gpweno_debug_poison(gpweno_ctx* c, long cell) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!c->state) return fail(c, GPWENO_ESTATE, "no state bound");
    if (cell < 0 || (long long)cell >= c->ncell) return fail(c, GPWENO_EINVAL, "cell %ld out of range", cell);
    c->shadow_ok = false;
    hipError_t e = gpw::launch_poison(c->state, c->nv, c->ncell, (long long)cell, user_stream(c));
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "poison launch: %s", hipGetErrorString(e));
    return GPWENO_OK;
}

const char* gpweno_last_error(const gpweno_ctx* c) { return c ? c->err.c_str() : g_tls_error.c_str(); }

void gpweno_destroy(gpweno_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(user_stream(c));  // NULL: the default stream
    if (c->own_stream) (void)hipStreamSynchronize(c->own_stream);
    drop_graph(c);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    ctl_release(c->device, c->d_ctl, c->h_ctl);
    delete c;
}

}  // extern "C"

// ===========================================================================
// Batched execution
// ===========================================================================
namespace {

constexpr int BATCH_MAX = 4096;
constexpr int BATCH_MAX_GROUPS = 64;
constexpr int DIR_PER_GROUP = 9;            // 3 stages x up to 3 directions
constexpr int STAGING = 4;                  // pinned staging buffers in the ring

// Captured batched steps of one group: its 3 ndim launches per step as a
// chain, for BATCH_GRAPH_STEPS[i] steps; a run of n steps replays them largest
// first (8 steps per graph launch instead of one: fewer host calls and gaps).
constexpr int BATCH_GRAPH_STEPS[2] = {8, 1};

struct StepGraph {
    hipGraphExec_t exec = nullptr;
    hipGraph_t src = nullptr;
    std::vector<hipGraphNode_t> nodes;      // kernel nodes in launch order
    std::vector<hipKernelNodeParams> params;
};

struct GroupGraph {
    StepGraph by_steps[2];                  // BATCH_GRAPH_STEPS[i] steps each
};

// Problems sharing one kernel instantiation per launch and one set of tables.
struct BatchGroup {
    int ndim = 0, R = 0, ik = 0, nc = 2;
    bool fp32 = false;
    bool bcg[3] = {false, false, false};    // the members' axis has a non-periodic side
    gpw::Tab<float> tabf[3];                // the group's tables (kernel arguments)
    gpw::Tab<double> tabd[3];
    std::vector<int> members;               // indices into the set
    long long blocks[3] = {0, 0, 0};        // logical blocks per direction
    size_t owner_off[3] = {0, 0, 0};        // element offsets into the owner table
    size_t desc_off[3][3] = {};             // [stage-1][dir] offsets into the descriptor table
};

// Kernel kind and tables of a group: the kernel instantiation of every launch
// (dimension, R, precision, indicator kind, flux-correction terms, periodic or
// general boundaries per axis) and the tables it receives, per axis. A problem
// runs the same kernels with the same arguments in a batch as alone, so its
// result is bitwise the same; a problem with non-square cells batches with
// those whose per-axis tables equal its own. A captured graph serves every set
// whose groups have the same kinds, in the same order.
bool same_kind(const BatchGroup& a, const BatchGroup& b) {
    if (a.ndim != b.ndim || a.R != b.R || a.fp32 != b.fp32 || a.ik != b.ik || a.nc != b.nc) return false;
    for (int d = 0; d < a.ndim; ++d) {
        if (a.bcg[d] != b.bcg[d]) return false;
        if (a.fp32 ? std::memcmp(&a.tabf[d], &b.tabf[d], sizeof(gpw::Tab<float>)) != 0
                   : std::memcmp(&a.tabd[d], &b.tabd[d], sizeof(gpw::Tab<double>)) != 0)
            return false;
    }
    return true;
}

size_t align_up(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

struct gpweno_batch {
    int device = 0;
    hipStream_t own_stream = nullptr;
    // the stream of the last set or run; a flag of its own, since the default
    // stream's handle is NULL
    hipStream_t last_stream = nullptr;
    bool last_used = false;
    std::vector<gpweno_ctx*> set;
    std::vector<BatchGroup> groups;
    // device work tables: per group and step position a BatchDir (fixed
    // addresses, which the captured graph's launches hold), the descriptors and
    // block owners they point to (grown as needed), the members' control blocks
    gpw::BatchDir* d_dir = nullptr;
    gpw::ProbDesc* d_desc = nullptr;
    size_t desc_cap = 0;
    unsigned short* d_owner = nullptr;
    size_t owner_cap = 0;
    gpw::Ctl** d_ctls = nullptr;
    gpw::BatchStatus* d_status = nullptr;
    gpw::BatchStatus* h_status = nullptr;
    // pinned staging ring for the stream-ordered table uploads
    unsigned char* staging[STAGING] = {};
    size_t staging_cap[STAGING] = {};
    hipEvent_t staging_done[STAGING] = {};
    bool staging_used[STAGING] = {};
    int staging_next = 0;
    // captured batched step: one graph per group (the group's launches of one
    // step, a chain), the kinds they were captured for, and each graph's kernel
    // nodes by step position with their parameters (their grids follow the set)
    std::vector<GroupGraph> graphs;
    std::vector<BatchGroup> graph_groups;
    bool nodes_ok = false;                   // every graph's nodes were found
    // with more than one group, each group's graph runs on a stream of its own,
    // forked from and joined back to the caller's stream
    hipStream_t group_stream[BATCH_MAX_GROUPS] = {};
    hipEvent_t group_join[BATCH_MAX_GROUPS] = {};
    hipEvent_t group_fork = nullptr;
    long long recaptures = 0;
    bool dirty = true;                       // the set changed since the grids were applied
    std::string err;
};

namespace {

int bfail(gpweno_batch* b, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    else g_tls_error = buf;
    return code;
}

#define BHIP_TRY(b, expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return bfail((b), GPWENO_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

void batch_drop_graph(gpweno_batch* b) {
    for (auto& gg : b->graphs)
        for (auto& sg : gg.by_steps) {
            if (sg.exec) (void)hipGraphExecDestroy(sg.exec);
            if (sg.src) (void)hipGraphDestroy(sg.src);
        }
    b->graphs.clear();
    b->graph_groups.clear();
    b->nodes_ok = false;
}

// One batched launch: step position k for group g (its work table entry
// d_dir[g * DIR_PER_GROUP + k]), with the given grid.
int batch_launch(gpweno_batch* b, int gi, const BatchGroup& g, int k, long long grid, hipStream_t s) {
    const int stage = k / g.ndim + 1, j = k % g.ndim, dir = sweep_dir(g.ndim, j);
    const bool fin = j == g.ndim - 1;
    const gpw::LaunchSel sel{dir, g.R, fin, g.ik, g.bcg[dir], g.nc, true};
    const gpw::BatchDir* D = b->d_dir + (size_t)gi * DIR_PER_GROUP + k;
    hipError_t e;
    if (g.fp32) {
        gpw::BatchArgs<float> a;
        std::memset(&a, 0, sizeof a);
        a.dir = D;
        a.first = j == 0;
        a.stage = stage;
        a.step_start = k == 0;
        a.tab = g.tabf[dir];
        e = gpw::launch_sweep(g.ndim, true, sel, &a, grid, s);
    } else {
        gpw::BatchArgs<double> a;
        std::memset(&a, 0, sizeof a);
        a.dir = D;
        a.first = j == 0;
        a.stage = stage;
        a.step_start = k == 0;
        a.tab = g.tabd[dir];
        e = gpw::launch_sweep(g.ndim, false, sel, &a, grid, s);
    }
    if (e != hipSuccess) return bfail(b, GPWENO_EHIP, "batched sweep launch: %s", hipGetErrorString(e));
    return GPWENO_OK;
}

// Grid of a batched launch: one block per logical block of the group's
// direction (one block for an empty group, which exits at once).
long long launch_grid(const BatchGroup& g, int k) {
    return std::max(1ll, g.members.empty() ? 0ll : g.blocks[sweep_dir(g.ndim, k % g.ndim)]);
}

// Whether the captured graph serves the current groups: the same kinds in the
// same order (its launches read the sets through the work tables; their grids
// are set per set by batch_update_grids).
bool graph_serves(const gpweno_batch* b) {
    if (b->graphs.empty() || b->graph_groups.size() != b->groups.size()) return false;
    for (size_t i = 0; i < b->groups.size(); ++i)
        if (!same_kind(b->graph_groups[i], b->groups[i])) return false;
    return true;
}

// Sets the grid of every launch of the instantiated graph to the current set's
// blocks (host-side; launches already enqueued keep the grids they had).
int batch_update_grids(gpweno_batch* b) {
    for (size_t gi = 0; gi < b->graphs.size(); ++gi) {
        const int nk = 3 * b->groups[gi].ndim;
        for (StepGraph& sg : b->graphs[gi].by_steps)
            for (size_t i = 0; i < sg.nodes.size(); ++i) {
                hipKernelNodeParams& p = sg.params[i];
                const long long gr = launch_grid(b->groups[gi], (int)(i % nk));
                if (gr > INT_MAX) return bfail(b, GPWENO_EINVAL, "batch too large");
                if ((long long)p.gridDim.x == gr) continue;
                p.gridDim.x = (unsigned)gr;
                hipError_t e = hipGraphExecKernelNodeSetParams(sg.exec, sg.nodes[i], &p);
                if (e != hipSuccess)
                    return bfail(b, GPWENO_EHIP, "hipGraphExecKernelNodeSetParams: %s", hipGetErrorString(e));
            }
    }
    return GPWENO_OK;
}

// Captures one group's launches of `steps` batched steps on the batch's own
// stream (a chain), instantiates it and finds its kernel nodes along the chain
// for the in-place grid updates (nodes_ok false if the runtime does not expose
// them; set changes then recapture).
int capture_steps(gpweno_batch* b, int gi, int steps, StepGraph& sg, bool& nodes_ok) {
    const BatchGroup& g = b->groups[gi];
    const int nk = 3 * g.ndim;
    BHIP_TRY(b, hipStreamBeginCapture(b->own_stream, hipStreamCaptureModeThreadLocal));
    int st = GPWENO_OK;
    for (int i = 0; i < steps * nk && !st; ++i) st = batch_launch(b, gi, g, i % nk, launch_grid(g, i % nk), b->own_stream);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(b->own_stream, &gr);
    if (st) {
        if (gr) (void)hipGraphDestroy(gr);
        return st;
    }
    if (e != hipSuccess) return bfail(b, GPWENO_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    sg.src = gr;
    e = hipGraphInstantiate(&sg.exec, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        sg.exec = nullptr;
        return bfail(b, GPWENO_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    std::vector<hipGraphNode_t> chain;
    size_t n = 1;
    hipGraphNode_t node = nullptr;
    bool ok = hipGraphGetRootNodes(gr, &node, &n) == hipSuccess && n == 1;
    while (ok && node) {
        chain.push_back(node);
        hipGraphNode_t next = nullptr;
        size_t m = 0;
        ok = hipGraphNodeGetDependentNodes(node, nullptr, &m) == hipSuccess && m <= 1;
        if (ok && m == 1) ok = hipGraphNodeGetDependentNodes(node, &next, &m) == hipSuccess;
        node = m == 1 ? next : nullptr;
    }
    ok = ok && (int)chain.size() == steps * nk;
    std::vector<hipKernelNodeParams> params(chain.size());
    for (size_t i = 0; ok && i < chain.size(); ++i) {
        hipGraphNodeType t;
        ok = hipGraphNodeGetType(chain[i], &t) == hipSuccess && t == hipGraphNodeTypeKernel &&
             hipGraphKernelNodeGetParams(chain[i], &params[i]) == hipSuccess &&
             (long long)params[i].gridDim.x == launch_grid(g, (int)(i % nk));
    }
    if (ok) {
        sg.nodes = std::move(chain);
        sg.params = std::move(params);
    }
    nodes_ok = nodes_ok && ok;
    return GPWENO_OK;
}

// Captures the batched step graphs of every group (BATCH_GRAPH_STEPS steps each).
int batch_capture(gpweno_batch* b) {
    // the old graphs may still be running (on the stream they were last
    // launched on, which waited for the group streams); an executable graph is
    // destroyed only once no launch of it is in flight
    if (!b->graphs.empty() && b->last_used) BHIP_TRY(b, hipStreamSynchronize(b->last_stream));
    batch_drop_graph(b);
    const size_t ng = b->groups.size();
    if (ng > 1) {
        if (!b->group_fork) BHIP_TRY(b, hipEventCreateWithFlags(&b->group_fork, hipEventDisableTiming));
        for (size_t gi = 0; gi < ng; ++gi) {
            if (!b->group_stream[gi])
                BHIP_TRY(b, hipStreamCreateWithFlags(&b->group_stream[gi], hipStreamNonBlocking));
            if (!b->group_join[gi]) BHIP_TRY(b, hipEventCreateWithFlags(&b->group_join[gi], hipEventDisableTiming));
        }
    }
    bool nodes_ok = true;
    b->graphs.resize(ng);
    for (size_t gi = 0; gi < ng; ++gi)
        for (int i = 0; i < 2; ++i) {
            int st = capture_steps(b, (int)gi, BATCH_GRAPH_STEPS[i], b->graphs[gi].by_steps[i], nodes_ok);
            if (st) {
                batch_drop_graph(b);
                return st;
            }
        }
    b->graph_groups = b->groups;
    b->nodes_ok = nodes_ok;
    ++b->recaptures;
    return GPWENO_OK;
}

// Replays nsteps batched steps of one group on stream gs, largest graphs first.
hipError_t replay_steps(const GroupGraph& gg, int nsteps, hipStream_t gs) {
    hipError_t e = hipSuccess;
    int left = nsteps;
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
        for (; left >= BATCH_GRAPH_STEPS[i] && e == hipSuccess; left -= BATCH_GRAPH_STEPS[i])
            e = hipGraphLaunch(gg.by_steps[i].exec, gs);
    return e;
}

// Enqueues nsteps batched steps on s: one group's graph directly on s; several
// groups each on a stream of its own (forked from s, all joined back into s),
// so that the groups' sweeps, which share no data, can run side by side.
int batch_launch_steps(gpweno_batch* b, int nsteps, hipStream_t s) {
    const size_t ng = b->graphs.size();
    if (ng == 1) {
        BHIP_TRY(b, replay_steps(b->graphs[0], nsteps, s));
        return GPWENO_OK;
    }
    BHIP_TRY(b, hipEventRecord(b->group_fork, s));
    hipError_t first = hipSuccess;
    for (size_t gi = 0; gi < ng; ++gi) {
        hipStream_t gs = b->group_stream[gi];
        hipError_t e = hipStreamWaitEvent(gs, b->group_fork, 0);
        if (e == hipSuccess) e = replay_steps(b->graphs[gi], nsteps, gs);
        // joined back even after a failure, so that s orders everything after it
        hipError_t e1 = hipEventRecord(b->group_join[gi], gs);
        if (e1 == hipSuccess) e1 = hipStreamWaitEvent(s, b->group_join[gi], 0);
        if (first == hipSuccess) first = e != hipSuccess ? e : e1;
    }
    if (first != hipSuccess) return bfail(b, GPWENO_EHIP, "batched step launch: %s", hipGetErrorString(first));
    return GPWENO_OK;
}

// Grows a device table to hold n elements. The old table may still be read by
// launches in flight, so growing waits for the stream first (capacities double,
// so this happens a logarithmic number of times).
template <typename T>
int grow(gpweno_batch* b, T** buf, size_t* cap, size_t n, hipStream_t s) {
    if (n <= *cap) return GPWENO_OK;
    size_t c = std::max<size_t>(2 * *cap, 1024);
    while (c < n) c *= 2;
    BHIP_TRY(b, hipStreamSynchronize(s));
    if (*buf) (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    BHIP_TRY(b, hipMalloc(buf, sizeof(T) * c));
    *cap = c;
    return GPWENO_OK;
}

}  // namespace

extern "C" {

int gpweno_set_end(gpweno_ctx* c, double t_final, long step_limit) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!c->state) return fail(c, GPWENO_ESTATE, "no state bound");
    hipError_t e = gpw::launch_set_run(c->d_ctl, t_final, step_limit < 0 ? LLONG_MAX : (long long)step_limit,
                                       user_stream(c));
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "set_run launch: %s", hipGetErrorString(e));
    c->shadow_ok = false;   // batched runs advance the state without this context
    return GPWENO_OK;
}

int gpweno_batch_create(gpweno_batch** out) {
    if (!out) return bfail(nullptr, GPWENO_EINVAL, "NULL output pointer");
    *out = nullptr;
    gpweno_batch* b = new (std::nothrow) gpweno_batch();
    if (!b) return bfail(nullptr, GPWENO_ENOMEM, "out of host memory");
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&b->d_dir, sizeof(gpw::BatchDir) * BATCH_MAX_GROUPS * DIR_PER_GROUP);
    if (e == hipSuccess) e = hipMalloc(&b->d_ctls, sizeof(gpw::Ctl*) * BATCH_MAX);
    if (e == hipSuccess) e = hipMalloc(&b->d_status, sizeof(gpw::BatchStatus) * BATCH_MAX);
    if (e == hipSuccess) e = hipHostMalloc(&b->h_status, sizeof(gpw::BatchStatus) * BATCH_MAX, hipHostMallocDefault);
    for (int i = 0; i < STAGING && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&b->staging_done[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_dir, 0, sizeof(gpw::BatchDir) * BATCH_MAX_GROUPS * DIR_PER_GROUP,
                                            b->own_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->own_stream);
    if (e != hipSuccess) {
        int code = bfail(nullptr, GPWENO_EHIP, "batch set-up: %s", hipGetErrorString(e));
        gpweno_batch_destroy(b);
        return code;
    }
    *out = b;
    return GPWENO_OK;
}

int gpweno_batch_set(gpweno_batch* b, gpweno_ctx* const* ctxs, int n, void* stream) {
    if (!b) return bfail(nullptr, GPWENO_EINVAL, "NULL batch");
    if (n < 0 || n > BATCH_MAX || (n > 0 && !ctxs)) return bfail(b, GPWENO_EINVAL, "need 0 <= n <= %d", BATCH_MAX);
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i] || !ctxs[i]->state) return bfail(b, GPWENO_EINVAL, "context %d is NULL or not bound", i);
        if (ctxs[i]->device != b->device) return bfail(b, GPWENO_EINVAL, "context %d is on another device", i);
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return bfail(b, GPWENO_EINVAL, "context %d repeated", i);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // work already enqueued on another stream must finish before this one
    // rewrites the tables it reads
    if (b->last_used && b->last_stream != s) BHIP_TRY(b, hipStreamSynchronize(b->last_stream));
    // groups, in the order their kinds first appear; kinds the captured graph
    // already has keep their place so that the graph keeps serving the set
    std::vector<BatchGroup> groups;
    for (const auto& g : b->graph_groups) {
        BatchGroup h = g;
        h.members.clear();
        groups.push_back(h);
    }
    for (int i = 0; i < n; ++i) {
        const gpweno_ctx* c = ctxs[i];
        BatchGroup cand;
        cand.ndim = c->grid.ndim;
        cand.R = c->R;
        cand.fp32 = c->opt.precision == GPWENO_FP32;
        cand.ik = indicator_kind(c);
        cand.nc = corr_terms(c);
        for (int d = 0; d < 3; ++d) {
            cand.bcg[d] = d < c->grid.ndim && general_bc(c->grid, d);
            cand.tabf[d] = c->tabf[d];
            cand.tabd[d] = c->tabd[d];
        }
        BatchGroup* g = nullptr;
        for (auto& h : groups)
            if (same_kind(h, cand)) {
                g = &h;
                break;
            }
        if (!g) {
            if ((int)groups.size() >= BATCH_MAX_GROUPS)
                return bfail(b, GPWENO_EINVAL, "more than %d kinds of problems in one batch", BATCH_MAX_GROUPS);
            groups.push_back(cand);
            g = &groups.back();
        }
        g->members.push_back(i);
    }
    // a kind with no member left keeps its place only while the graph has it;
    // drop empty groups at the end, and every empty group if the graph must be
    // recaptured anyway
    while (!groups.empty() && groups.back().members.empty()) groups.pop_back();
    // descriptors, block owners and the work-table entries
    std::vector<gpw::ProbDesc> desc;
    std::vector<unsigned short> owner;
    for (auto& g : groups) {
        for (int dir = 0; dir < g.ndim; ++dir) {
            g.owner_off[dir] = owner.size();
            long long total = 0;
            std::vector<long long> nblk(g.members.size()), b0(g.members.size());
            for (size_t j = 0; j < g.members.size(); ++j) {
                const gpweno_ctx* c = ctxs[g.members[j]];
                int nn[3] = {c->grid.n[0], c->grid.n[1], c->grid.n[2]};
                const int nseg = (nn[dir] + run_cells(c) - 1) / run_cells(c);
                nblk[j] = gpw::sweep_blocks(g.ndim, dir, g.fp32, nn, nseg);
                b0[j] = total;
                total += nblk[j];
                for (long long q = 0; q < nblk[j]; ++q) owner.push_back((unsigned short)j);
            }
            if (total > INT_MAX) return bfail(b, GPWENO_EINVAL, "batch too large");
            g.blocks[dir] = total;
            for (int stage = 1; stage <= 3; ++stage) {
                g.desc_off[stage - 1][dir] = desc.size();
                for (size_t j = 0; j < g.members.size(); ++j) {
                    gpweno_ctx* c = ctxs[g.members[j]];
                    gpw::ProbDesc P;
                    std::memset(&P, 0, sizeof P);
                    const double* ins[3] = {c->state, c->U1, c->U2};
                    double* outs[3] = {c->U1, c->U2, c->state};
                    P.U = ins[stage - 1];
                    P.Un = c->state;
                    P.dU = c->dU;
                    P.Uout = outs[stage - 1];
                    P.ctl = c->d_ctl;
                    for (int d = 0; d < 3; ++d) P.n[d] = c->grid.n[d];
                    P.nseg = (c->grid.n[dir] + run_cells(c) - 1) / run_cells(c);
                    P.ncell = c->ncell;
                    P.inv_dx = 1.0 / c->dx[dir];
                    for (int d = 0; d < 3; ++d) P.inv_dx_all[d] = d < c->grid.ndim ? 1.0 / c->dx[d] : 0.0;
                    P.gamma = c->gamma;
                    P.inv_gm1 = 1.0 / (c->gamma - 1.0);
                    P.positivity = c->opt.positivity_fallback ? 1 : 0;
                    P.bc[0] = c->grid.bc[dir][0];
                    P.bc[1] = c->grid.bc[dir][1];
                    P.nblk = (unsigned)nblk[j];
                    P.block0 = b0[j];
                    desc.push_back(P);
                }
            }
        }
    }
    int st;
    if ((st = grow(b, &b->d_desc, &b->desc_cap, desc.size(), s))) return st;
    if ((st = grow(b, &b->d_owner, &b->owner_cap, owner.size(), s))) return st;
    std::vector<gpw::BatchDir> dirs((size_t)BATCH_MAX_GROUPS * DIR_PER_GROUP);
    std::memset(dirs.data(), 0, sizeof(gpw::BatchDir) * dirs.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const BatchGroup& g = groups[gi];
        for (int k = 0; k < 3 * g.ndim; ++k) {
            const int stage = k / g.ndim + 1, dir = sweep_dir(g.ndim, k % g.ndim);
            gpw::BatchDir& D = dirs[gi * DIR_PER_GROUP + k];
            D.probs = b->d_desc + g.desc_off[stage - 1][dir];
            D.owner = b->d_owner + g.owner_off[dir];
            D.nblocks = g.members.empty() ? 0 : g.blocks[dir];
        }
    }
    std::vector<gpw::Ctl*> ctls(n);
    for (int i = 0; i < n; ++i) ctls[i] = ctxs[i]->d_ctl;
    // stage everything in one pinned buffer of the ring and copy it in stream
    // order: launches enqueued before this call still read the old tables
    const size_t o_desc = 0, o_owner = align_up(o_desc + sizeof(gpw::ProbDesc) * desc.size());
    const size_t o_dir = align_up(o_owner + sizeof(unsigned short) * owner.size());
    const size_t o_ctl = align_up(o_dir + sizeof(gpw::BatchDir) * dirs.size());
    const size_t bytes = align_up(o_ctl + sizeof(gpw::Ctl*) * ctls.size());
    const int slot = b->staging_next;
    b->staging_next = (slot + 1) % STAGING;
    if (b->staging_used[slot]) BHIP_TRY(b, hipEventSynchronize(b->staging_done[slot]));
    if (bytes > b->staging_cap[slot]) {
        if (b->staging[slot]) (void)hipHostFree(b->staging[slot]);
        b->staging[slot] = nullptr;
        b->staging_cap[slot] = 0;
        const size_t c = std::max(bytes, (size_t)1 << 16);
        BHIP_TRY(b, hipHostMalloc(&b->staging[slot], c, hipHostMallocDefault));
        b->staging_cap[slot] = c;
    }
    unsigned char* h = b->staging[slot];
    if (!desc.empty()) std::memcpy(h + o_desc, desc.data(), sizeof(gpw::ProbDesc) * desc.size());
    if (!owner.empty()) std::memcpy(h + o_owner, owner.data(), sizeof(unsigned short) * owner.size());
    std::memcpy(h + o_dir, dirs.data(), sizeof(gpw::BatchDir) * dirs.size());
    if (n) std::memcpy(h + o_ctl, ctls.data(), sizeof(gpw::Ctl*) * ctls.size());
    if (!desc.empty())
        BHIP_TRY(b, hipMemcpyAsync(b->d_desc, h + o_desc, sizeof(gpw::ProbDesc) * desc.size(), hipMemcpyHostToDevice, s));
    if (!owner.empty())
        BHIP_TRY(b, hipMemcpyAsync(b->d_owner, h + o_owner, sizeof(unsigned short) * owner.size(),
                                   hipMemcpyHostToDevice, s));
    BHIP_TRY(b, hipMemcpyAsync(b->d_dir, h + o_dir, sizeof(gpw::BatchDir) * dirs.size(), hipMemcpyHostToDevice, s));
    if (n) BHIP_TRY(b, hipMemcpyAsync(b->d_ctls, h + o_ctl, sizeof(gpw::Ctl*) * n, hipMemcpyHostToDevice, s));
    BHIP_TRY(b, hipEventRecord(b->staging_done[slot], s));
    b->staging_used[slot] = true;
    b->set.assign(ctxs, ctxs + n);
    b->groups = std::move(groups);
    b->last_stream = s;
    b->last_used = true;
    b->dirty = true;
    return GPWENO_OK;
}

int gpweno_batch_run(gpweno_batch* b, int nsteps, void* stream) {
    if (!b) return bfail(nullptr, GPWENO_EINVAL, "NULL batch");
    if (nsteps < 1) return bfail(b, GPWENO_EINVAL, "nsteps must be >= 1");
    if (b->set.empty()) return GPWENO_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->last_used && b->last_stream != s) BHIP_TRY(b, hipStreamSynchronize(b->last_stream));
    if (graph_serves(b) && (!b->dirty || b->nodes_ok)) {
        if (b->dirty) {
            int st = batch_update_grids(b);
            if (st) return st;
        }
    } else {
        // a new kind of problem: capture anew with only the kinds the set has
        // (the graph holds no table address but the fixed work-table entries,
        // so a set change within the captured kinds never needs this)
        std::vector<BatchGroup> kept;
        for (auto& g : b->groups)
            if (!g.members.empty()) kept.push_back(g);
        if (kept.size() != b->groups.size()) {
            std::vector<gpweno_ctx*> set = b->set;
            b->graph_groups.clear();
            b->groups.clear();
            int st = gpweno_batch_set(b, set.data(), (int)set.size(), stream);
            if (st) return st;
        }
        int st = batch_capture(b);
        if (st) return st;
    }
    b->dirty = false;
    int st = batch_launch_steps(b, nsteps, s);
    b->last_stream = s;
    b->last_used = true;
    if (st) return st;
    return GPWENO_OK;
}

int gpweno_batch_status(gpweno_batch* b, double* t, double* dt, long* nsteps, int* err, void* stream) {
    if (!b) return bfail(nullptr, GPWENO_EINVAL, "NULL batch");
    const int n = (int)b->set.size();
    if (n == 0) return GPWENO_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // steps enqueued on another stream must have run before their status is read
    if (b->last_used && b->last_stream != s) BHIP_TRY(b, hipStreamSynchronize(b->last_stream));
    hipError_t e = gpw::launch_gather_status(b->d_ctls, n, b->d_status, s);
    if (e != hipSuccess) return bfail(b, GPWENO_EHIP, "status launch: %s", hipGetErrorString(e));
    BHIP_TRY(b, hipMemcpyAsync(b->h_status, b->d_status, sizeof(gpw::BatchStatus) * n, hipMemcpyDeviceToHost, s));
    BHIP_TRY(b, hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i) {
        if (t) t[i] = b->h_status[i].t;
        if (dt) dt[i] = b->h_status[i].dt;
        if (nsteps) nsteps[i] = (long)b->h_status[i].nsteps;
        if (err) err[i] = b->h_status[i].err;
    }
    return GPWENO_OK;
}

long gpweno_batch_captures(const gpweno_batch* b) { return b ? (long)b->recaptures : -1; }

void gpweno_batch_destroy(gpweno_batch* b) {
    if (!b) return;
    if (b->last_used) (void)hipStreamSynchronize(b->last_stream);
    if (b->own_stream) (void)hipStreamSynchronize(b->own_stream);
    for (int i = 0; i < BATCH_MAX_GROUPS; ++i)
        if (b->group_stream[i]) (void)hipStreamSynchronize(b->group_stream[i]);
    batch_drop_graph(b);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_owner) (void)hipFree(b->d_owner);
    if (b->d_dir) (void)hipFree(b->d_dir);
    if (b->d_ctls) (void)hipFree(b->d_ctls);
    if (b->d_status) (void)hipFree(b->d_status);
    if (b->h_status) (void)hipHostFree(b->h_status);
    for (int i = 0; i < STAGING; ++i) {
        if (b->staging[i]) (void)hipHostFree(b->staging[i]);
        if (b->staging_done[i]) (void)hipEventDestroy(b->staging_done[i]);
    }
    for (int i = 0; i < BATCH_MAX_GROUPS; ++i) {
        if (b->group_stream[i]) (void)hipStreamDestroy(b->group_stream[i]);
        if (b->group_join[i]) (void)hipEventDestroy(b->group_join[i]);
    }
    if (b->group_fork) (void)hipEventDestroy(b->group_fork);
    if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
    delete b;
}

const char* gpweno_batch_last_error(const gpweno_batch* b) { return b ? b->err.c_str() : g_tls_error.c_str(); }

}  // extern "C"

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
// captured HIP graph of several steps and synchronises once per replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/gpweno.h"
#include "gp_tables.h"
#include "gpweno_kernels.h"

namespace {

constexpr int TOUT = 58;            // cells produced per 64-cell run
constexpr int NPART = 1024;         // partial sums of the conservation reduction
constexpr int GRAPH_STEPS = 32;     // steps per captured graph

thread_local std::string g_tls_error = "";

}  // namespace

struct gpweno_ctx {
    gpweno_grid grid;
    int R;
    double ell, sigma, gamma;
    double dx[3];
    long long ncell;
    int nv;
    gpweno_options opt;
    GpTablesF64 tab64[3];
    gpw::Tab<double> tabd[3];
    gpw::Tab<float> tabf[3];
    int device;
    gpw::Ctl* d_ctl = nullptr;
    gpw::Ctl* h_ctl = nullptr;      // pinned mirror
    hipStream_t own_stream = nullptr;
    double* state = nullptr;
    double* U1 = nullptr;
    double* U2 = nullptr;
    double* dU = nullptr;
    double* partials = nullptr;
    hipGraphExec_t graph = nullptr;
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
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
}

template <typename Real>
gpw::SweepArgs<Real> base_args(const gpweno_ctx* c, int dir) {
    gpw::SweepArgs<Real> a;
    std::memset(&a, 0, sizeof a);
    for (int d = 0; d < 3; ++d) a.n[d] = d < c->grid.ndim ? c->grid.n[d] : 1;
    a.nseg = (a.n[dir] + TOUT - 1) / TOUT;
    a.ncell = c->ncell;
    a.inv_dx = 1.0 / c->dx[dir];
    for (int d = 0; d < 3; ++d) a.inv_dx_all[d] = d < c->grid.ndim ? 1.0 / c->dx[d] : 0.0;
    a.gamma = c->gamma;
    a.positivity = c->opt.positivity_fallback ? 1 : 0;
    a.ctl = c->d_ctl;
    if constexpr (sizeof(Real) == 8) a.tab = c->tabd[dir];
    else a.tab = c->tabf[dir];
    return a;
}

// One sweep launch (direction dir) in the configured precision.
int launch(gpweno_ctx* c, int dir, const double* in, const double* un, double* acc, double* out, int stage,
           bool fin, bool first, bool step_start, hipStream_t s) {
    const bool fp32 = c->opt.precision == GPWENO_FP32;
    hipError_t e;
    if (fp32) {
        auto a = base_args<float>(c, dir);
        a.U = in; a.Un = un; a.dU = acc; a.Uout = out;
        a.first = first; a.stage = stage; a.step_start = step_start;
        e = gpw::launch_sweep(c->grid.ndim, dir, c->R, true, fin, &a, s);
    } else {
        auto a = base_args<double>(c, dir);
        a.U = in; a.Un = un; a.dU = acc; a.Uout = out;
        a.first = first; a.stage = stage; a.step_start = step_start;
        e = gpw::launch_sweep(c->grid.ndim, dir, c->R, false, fin, &a, s);
    }
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "sweep launch (dir %d): %s", dir, hipGetErrorString(e));
    return GPWENO_OK;
}

// The k-th launch of a step: stage k / ndim + 1, direction k % ndim.
int launch_step_kernel(gpweno_ctx* c, int k, hipStream_t s) {
    const int ndim = c->grid.ndim;
    const int stage = k / ndim + 1, dir = k % ndim;
    const double* ins[3] = {c->state, c->U1, c->U2};
    double* outs[3] = {c->U1, c->U2, c->state};
    return launch(c, dir, ins[stage - 1], c->state, c->dU, outs[stage - 1], stage, dir == ndim - 1, dir == 0,
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

// Captures GRAPH_STEPS steps on the private stream (capture records, it does
// not execute); the graph is launched on the caller's stream.
int ensure_graph(gpweno_ctx* c) {
    if (c->graph) return GPWENO_OK;
    hipStream_t s = c->own_stream;
    HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int st = GPWENO_OK;
    for (int k = 0; k < GRAPH_STEPS && st == GPWENO_OK; ++k) st = enqueue_step(c, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->graph = nullptr;
        return fail(c, GPWENO_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return GPWENO_OK;
}

bool valid_options(const gpweno_options* o) {
    return o && (o->precision == GPWENO_FP64 || o->precision == GPWENO_FP32) && o->cfl > 0 &&
           std::isfinite(o->cfl) && o->fixed_dt >= 0 && std::isfinite(o->fixed_dt);
}

template <typename Real>
void fill_tab(gpw::Tab<Real>& t, const GpTablesF64& s) {
    for (int m = 0; m < 4; ++m) {
        t.gp[m] = (Real)s.gam_plus[m];
        t.gm[m] = (Real)s.gam_minus[m];
        for (int j = 0; j < 4; ++j) {
            t.wp[m][j] = (Real)s.w_plus[m][j];
            t.wm[m][j] = (Real)s.w_minus[m][j];
            t.P[m][j] = (Real)s.P[m][j];
        }
    }
}

}  // namespace

extern "C" {

int gpweno_compute_tables(int R, double ell_over_dx, double sigma_over_dx, double* w_plus, double* w_minus,
                          double* gam_plus, double* gam_minus, double* P) {
    if (R < 1 || R > 3) return fail(nullptr, GPWENO_EINVAL, "R must be 1, 2 or 3 (got %d)", R);
    if (!(ell_over_dx > 0) || !std::isfinite(ell_over_dx) || !(sigma_over_dx > 0) || !std::isfinite(sigma_over_dx))
        return fail(nullptr, GPWENO_EINVAL, "length scales must be positive and finite");
    GpTablesF64 t;
    int st = gpw_build_tables(R, ell_over_dx, sigma_over_dx, &t);
    if (st) return fail(nullptr, GPWENO_EINVAL, "table construction failed (%d)", st);
    if (w_plus) std::memcpy(w_plus, t.w_plus, sizeof t.w_plus);
    if (w_minus) std::memcpy(w_minus, t.w_minus, sizeof t.w_minus);
    if (gam_plus) std::memcpy(gam_plus, t.gam_plus, sizeof t.gam_plus);
    if (gam_minus) std::memcpy(gam_minus, t.gam_minus, sizeof t.gam_minus);
    if (P) std::memcpy(P, t.P, sizeof t.P);
    return GPWENO_OK;
}

int gpweno_init(const gpweno_grid* grid, int R, double ell, double sigma, double gamma, gpweno_ctx** out) {
    if (!grid || !out) return fail(nullptr, GPWENO_EINVAL, "NULL grid or output pointer");
    *out = nullptr;
    if (grid->ndim < 1 || grid->ndim > 3) return fail(nullptr, GPWENO_EINVAL, "ndim must be 1, 2 or 3");
    if (R < 1 || R > 3) return fail(nullptr, GPWENO_EINVAL, "R must be 1, 2 or 3 (got %d)", R);
    if (!(gamma > 1.0) || !std::isfinite(gamma)) return fail(nullptr, GPWENO_EINVAL, "gamma must be > 1");
    if (!(ell > 0) || !std::isfinite(ell)) return fail(nullptr, GPWENO_EINVAL, "ell must be positive");
    gpweno_ctx* c = new (std::nothrow) gpweno_ctx();
    if (!c) return fail(nullptr, GPWENO_ENOMEM, "out of host memory");
    c->grid = *grid;
    c->R = R;
    c->ell = ell;
    c->sigma = sigma;
    c->gamma = gamma;
    c->nv = 2 + grid->ndim;
    c->ncell = 1;
    for (int d = 0; d < 3; ++d) {
        if (d >= grid->ndim) {
            c->grid.n[d] = 1;
            c->dx[d] = 1.0;
            continue;
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
        int st = gpw_build_tables(R, ell / c->dx[d], sigma / c->dx[d], &c->tab64[d]);
        if (st) {
            delete c;
            return fail(nullptr, GPWENO_EINVAL, "table construction failed on axis %d (%d)", d, st);
        }
        fill_tab(c->tabd[d], c->tab64[d]);
        fill_tab(c->tabf[d], c->tab64[d]);
    }
    if (c->ncell > (1ll << 40)) {
        delete c;
        return fail(nullptr, GPWENO_EINVAL, "grid too large");
    }
    c->opt.precision = GPWENO_FP64;
    c->opt.cfl = 0.4;
    c->opt.fixed_dt = 0.0;
    c->opt.positivity_fallback = 0;
    c->opt.stream = nullptr;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipMalloc(&c->d_ctl, sizeof(gpw::Ctl));
    if (e == hipSuccess) e = hipHostMalloc(&c->h_ctl, sizeof(gpw::Ctl), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemset(c->d_ctl, 0, sizeof(gpw::Ctl));
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
    const bool changes_graph = o->precision != c->opt.precision ||
                               o->positivity_fallback != c->opt.positivity_fallback || o->stream != c->opt.stream;
    const bool changes_rule = o->cfl != c->opt.cfl || o->fixed_dt != c->opt.fixed_dt;
    c->opt = *o;
    if (changes_graph) drop_graph(c);
    if (changes_rule && c->state) {
        // the CFL number and fixed dt live in the control block
        if (read_ctl(c, user_stream(c))) return GPWENO_EHIP;
        hipError_t e = gpw::launch_set_time(c->d_ctl, c->h_ctl->t, c->h_ctl->nsteps, c->opt.cfl, c->opt.fixed_dt,
                                            user_stream(c));
        if (e != hipSuccess) return fail(c, GPWENO_EHIP, "set_time launch: %s", hipGetErrorString(e));
        const int n[3] = {c->grid.n[0], c->grid.n[1], c->grid.n[2]};
        const double ix[3] = {1.0 / c->dx[0], c->grid.ndim > 1 ? 1.0 / c->dx[1] : 0.0,
                              c->grid.ndim > 2 ? 1.0 / c->dx[2] : 0.0};
        e = gpw::launch_speed(c->grid.ndim, c->state, c->ncell, n, ix, c->gamma, c->d_ctl, user_stream(c));
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
    const int n[3] = {c->grid.n[0], c->grid.n[1], c->grid.n[2]};
    const double ix[3] = {1.0 / c->dx[0], c->grid.ndim > 1 ? 1.0 / c->dx[1] : 0.0,
                          c->grid.ndim > 2 ? 1.0 / c->dx[2] : 0.0};
    e = gpw::launch_speed(c->grid.ndim, c->state, c->ncell, n, ix, c->gamma, c->d_ctl, s);
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "speed launch: %s", hipGetErrorString(e));
    return GPWENO_OK;
}

int gpweno_bind(gpweno_ctx* c, double* d_state, void* d_workspace) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!d_state || !d_workspace) return fail(c, GPWENO_EINVAL, "NULL state or workspace");
    if (((uintptr_t)d_state & 7) || ((uintptr_t)d_workspace & 255))
        return fail(c, GPWENO_EINVAL, "state must be 8-byte and workspace 256-byte aligned");
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

int gpweno_step(gpweno_ctx* c, double t_final) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!c->state) return fail(c, GPWENO_ESTATE, "no state bound");
    hipStream_t s = user_stream(c);
    hipError_t e = gpw::launch_set_run(c->d_ctl, t_final, LLONG_MAX, s);
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "set_run launch: %s", hipGetErrorString(e));
    return enqueue_step(c, s);
}

int gpweno_run(gpweno_ctx* c, double t_final, long max_steps, long* nsteps_out, double* t_out) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    if (!c->state) return fail(c, GPWENO_ESTATE, "no state bound");
    if (nsteps_out) *nsteps_out = 0;
    hipStream_t s = user_stream(c);
    int st = read_ctl(c, s);
    if (st) return st;
    if ((st = check_err(c))) return st;
    const long long start = c->h_ctl->nsteps;
    const long long limit = max_steps < 0 ? LLONG_MAX : start + max_steps;
    hipError_t e = gpw::launch_set_run(c->d_ctl, t_final, limit, s);
    if (e != hipSuccess) return fail(c, GPWENO_EHIP, "set_run launch: %s", hipGetErrorString(e));
    while (c->h_ctl->t < t_final && c->h_ctl->nsteps < limit) {
        if ((st = ensure_graph(c))) return st;
        HIP_TRY(c, hipGraphLaunch(c->graph, s));
        if ((st = read_ctl(c, s))) return st;
        if ((st = check_err(c))) break;
    }
    if (nsteps_out) *nsteps_out = (long)(c->h_ctl->nsteps - start);
    if (t_out) *t_out = c->h_ctl->t;
    return st;
}

int gpweno_get_time(gpweno_ctx* c, double* t, double* dt, long* nsteps) {
    if (!c) return fail(nullptr, GPWENO_EINVAL, "NULL context");
    int st = read_ctl(c, user_stream(c));
    if (st) return st;
    if (t) *t = c->h_ctl->t;
    if (dt) *dt = c->h_ctl->dt;
    if (nsteps) *nsteps = (long)c->h_ctl->nsteps;
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

const char* gpweno_last_error(const gpweno_ctx* c) { return c ? c->err.c_str() : g_tls_error.c_str(); }

void gpweno_destroy(gpweno_ctx* c) {
    if (!c) return;
    if (c->opt.stream) (void)hipStreamSynchronize(user_stream(c));
    if (c->own_stream) (void)hipStreamSynchronize(c->own_stream);
    drop_graph(c);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    if (c->d_ctl) (void)hipFree(c->d_ctl);
    if (c->h_ctl) (void)hipHostFree(c->h_ctl);
    delete c;
}

}  // extern "C"

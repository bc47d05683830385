// Control, CFL-speed and conservation kernels, and the launch dispatch of the
// sweeps (whose instances live in gpweno_sweep_<ndim>d_<precision>.hip).
#include "gpweno_sweep.h"

namespace gpw {

// sweep instances, one translation unit per dimension and precision
hipError_t launch_sweep_1d_f32(const LaunchSel& k, const void* args, long long blocks, hipStream_t s);
hipError_t launch_sweep_1d_f64(const LaunchSel& k, const void* args, long long blocks, hipStream_t s);
hipError_t launch_sweep_2d_f32(const LaunchSel& k, const void* args, long long blocks, hipStream_t s);
hipError_t launch_sweep_2d_f64(const LaunchSel& k, const void* args, long long blocks, hipStream_t s);
hipError_t launch_sweep_3d_f32(const LaunchSel& k, const void* args, long long blocks, hipStream_t s);
hipError_t launch_sweep_3d_f64(const LaunchSel& k, const void* args, long long blocks, hipStream_t s);

// ---------------------------------------------------------------------------
// Time-step control and reductions
// ---------------------------------------------------------------------------

__global__ void set_run_kernel(Ctl* c, double t_final, long long step_limit) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    c->t_final = t_final;
    c->step_limit = step_limit;
}

__global__ void set_run_rel_kernel(Ctl* c, double t_final, long long max_steps) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const StepRec& r = c->rec[0].nsteps > c->rec[1].nsteps ? c->rec[0] : c->rec[1];
    c->t_final = t_final;
    c->run_start = r.nsteps;
    c->run_t0 = r.t;
    c->step_limit = max_steps < 0 || max_steps > LLONG_MAX - r.nsteps ? LLONG_MAX : r.nsteps + max_steps;
}

__global__ void set_time_kernel(Ctl* c, double t, long long nsteps, double cfl, double fixed_dt) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    c->rec[0].t = t;
    c->rec[0].dt = 0.0;
    c->rec[0].nsteps = nsteps;
    c->rec[1].t = t;
    c->rec[1].dt = 0.0;
    c->rec[1].nsteps = nsteps - 1;
    c->started = -1;
    c->cfl = cfl;
    c->fixed_dt = fixed_dt;
    c->err = 0;
    c->bad_cell = LLONG_MAX;
    c->dt_step[0] = 0.0;
    c->dt_step[1] = 0.0;
    for (int x = 0; x < 8; ++x) {
        c->xcd[x].speed[0] = 0ull;
        c->xcd[x].speed[1] = 0ull;
    }
}

// CFL speed max_i sum_d (|u_d| + c)/dx_d of a state, with the physical check.
// Each cell's speed is formed by cell_speed, the function the finishing sweep
// of stage 3 applies to the state it writes, so a state gets the same dt here
// (after gpweno_bind / gpweno_set_time) as when a step produced it: a run
// resumed from a saved state retraces the uninterrupted run bit for bit.
template <int NDIM>
__global__ void __launch_bounds__(256) speed_kernel(const double* __restrict__ U, long long ncell, double ix0,
                                                    double ix1, double ix2, double gamma, Ctl* ctl) {
    constexpr int NV = 2 + NDIM;
    __shared__ unsigned long long sred[4];
    const double ix[3] = {ix0, ix1, ix2};
    unsigned long long smax = 0;
    for (long long cell = blockIdx.x * (long long)blockDim.x + threadIdx.x; cell < ncell;
         cell += (long long)gridDim.x * blockDim.x) {
        double o[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) o[k] = U[k * ncell + cell];
        bool ok;
        const double s = cell_speed<NDIM>(o, gamma, ix, ok, true);
        if (!ok) {
            atomicOr(&ctl->err, 1);
            atomicMin(&ctl->bad_cell, cell);
        }
        const unsigned long long bits = (unsigned long long)__double_as_longlong(s);
        smax = bits > smax ? bits : smax;
    }
    smax = wave_max_u64(smax);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = smax;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = sred[0];
        for (int i = 1; i < 4; ++i) m = sred[i] > m ? sred[i] : m;
        const long long n = ctl->rec[0].nsteps > ctl->rec[1].nsteps ? ctl->rec[0].nsteps : ctl->rec[1].nsteps;
        atomicMax(&ctl->xcd[blockIdx.x & 7u].speed[n & 1], m);
    }
}

__global__ void step_prep_kernel(Ctl* c, double cfl, double fixed_dt, double t_final) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const long long n = c->rec[0].nsteps > c->rec[1].nsteps ? c->rec[0].nsteps : c->rec[1].nsteps;
    c->cfl = cfl;
    c->fixed_dt = fixed_dt;
    c->t_final = t_final;
    c->step_limit = LLONG_MAX;
    for (int x = 0; x < 8; ++x) c->xcd[x].speed[n & 1] = 0ull;
}

// Test hook: density and total energy of one cell set to -1.
__global__ void poison_kernel(double* U, int nv, long long ncell, long long cell) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    U[cell] = -1.0;
    U[(long long)(nv - 1) * ncell + cell] = -1.0;
}

// Deterministic float64 sums: fixed per-thread strides, fixed tree per block,
// then one block adds the per-block partials in index order.
__global__ void __launch_bounds__(256) sums_partial_kernel(const double* __restrict__ U, long long ncell, int nv,
                                                           double* __restrict__ partials) {
    __shared__ double sh[256];
    for (int k = 0; k < nv; ++k) {
        double acc = 0.0;
        for (long long i = blockIdx.x * 256ll + threadIdx.x; i < ncell; i += (long long)gridDim.x * 256)
            acc += U[k * ncell + i];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) partials[k * gridDim.x + blockIdx.x] = sh[0];
        __syncthreads();
    }
}

__global__ void sums_final_kernel(const double* __restrict__ partials, int npart, int nv, Ctl* ctl) {
    const int k = threadIdx.x;
    if (k >= nv) return;
    double acc = 0.0;
    for (int b = 0; b < npart; ++b) acc += partials[k * npart + b];
    ctl->sums[k] = acc;
}


hipError_t launch_sweep(int ndim, bool fp32, const LaunchSel& k, const void* args, long long blocks, hipStream_t s) {
    switch (ndim) {
        case 1: return fp32 ? launch_sweep_1d_f32(k, args, blocks, s) : launch_sweep_1d_f64(k, args, blocks, s);
        case 2: return fp32 ? launch_sweep_2d_f32(k, args, blocks, s) : launch_sweep_2d_f64(k, args, blocks, s);
        case 3: return fp32 ? launch_sweep_3d_f32(k, args, blocks, s) : launch_sweep_3d_f64(k, args, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

// ---- batched launches --------------------------------------------------------
long long sweep_blocks(int ndim, int dir, bool fp32, const int n[3], int nseg) {
    const int wpb = sweep_wpb(ndim, dir, fp32);
    long long groups;
    if (dir == 0) groups = ((long long)n[1] * n[2] + wpb - 1) / wpb;
    else groups = (long long)((n[0] + wpb - 1) / wpb) * (dir == 1 ? n[2] : n[1]);
    return groups * nseg;
}

// Copies the step state of every problem of a batch into a compact array.
__global__ void gather_status_kernel(Ctl* const* ctls, int nprob, BatchStatus* out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob) return;
    const Ctl* c = ctls[p];
    const StepRec& r = c->rec[0].nsteps > c->rec[1].nsteps ? c->rec[0] : c->rec[1];
    out[p].t = r.t;
    out[p].dt = r.dt;
    out[p].nsteps = r.nsteps;
    out[p].err = c->err;
    out[p].pad = 0;
}

hipError_t launch_gather_status(Ctl* const* ctls, int nprob, BatchStatus* out, hipStream_t s) {
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_status_kernel, dim3((nprob + 63) / 64), dim3(64), 0, s, ctls, nprob, out);
    return hipGetLastError();
}

hipError_t launch_set_run(Ctl* ctl, double t_final, long long step_limit, hipStream_t s) {
    hipLaunchKernelGGL(set_run_kernel, dim3(1), dim3(64), 0, s, ctl, t_final, step_limit);
    return hipGetLastError();
}

hipError_t launch_set_run_rel(Ctl* ctl, double t_final, long long max_steps, hipStream_t s) {
    hipLaunchKernelGGL(set_run_rel_kernel, dim3(1), dim3(64), 0, s, ctl, t_final, max_steps);
    return hipGetLastError();
}

hipError_t launch_set_time(Ctl* ctl, double t, long long nsteps, double cfl, double fixed_dt, hipStream_t s) {
    hipLaunchKernelGGL(set_time_kernel, dim3(1), dim3(64), 0, s, ctl, t, nsteps, cfl, fixed_dt);
    return hipGetLastError();
}

hipError_t launch_speed(int ndim, const double* U, long long ncell, const double inv_dx[3], double gamma, Ctl* ctl,
                        hipStream_t s) {
    long long blocks = (ncell + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    const dim3 g((unsigned)blocks), b(256);
    switch (ndim) {
        case 1: hipLaunchKernelGGL(speed_kernel<1>, g, b, 0, s, U, ncell, inv_dx[0], inv_dx[1], inv_dx[2], gamma, ctl); break;
        case 2: hipLaunchKernelGGL(speed_kernel<2>, g, b, 0, s, U, ncell, inv_dx[0], inv_dx[1], inv_dx[2], gamma, ctl); break;
        case 3: hipLaunchKernelGGL(speed_kernel<3>, g, b, 0, s, U, ncell, inv_dx[0], inv_dx[1], inv_dx[2], gamma, ctl); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step_prep(Ctl* ctl, double cfl, double fixed_dt, double t_final, hipStream_t s) {
    hipLaunchKernelGGL(step_prep_kernel, dim3(1), dim3(64), 0, s, ctl, cfl, fixed_dt, t_final);
    return hipGetLastError();
}

hipError_t launch_poison(double* U, int nv, long long ncell, long long cell, hipStream_t s) {
    hipLaunchKernelGGL(poison_kernel, dim3(1), dim3(64), 0, s, U, nv, ncell, cell);
    return hipGetLastError();
}

hipError_t launch_sums(int nv, const double* U, long long ncell, double* partials, int npart, Ctl* ctl,
                       hipStream_t s) {
    hipLaunchKernelGGL(sums_partial_kernel, dim3(npart), dim3(256), 0, s, U, ncell, nv, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sums_final_kernel, dim3(1), dim3(64), 0, s, partials, npart, nv, ctl);
    return hipGetLastError();
}

}  // namespace gpw


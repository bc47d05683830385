// Device-side data shared by the kernels and the host API of libgpweno.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpw {

constexpr int WAVE = 64;

// A sweep maps a run of 64 consecutive cells of a pencil onto the lanes of a
// wave. With NC terms of the flux correction (face fluxes NC faces either side
// of a face, plus one face for the difference), lanes run_left(NC) ..
// run_left(NC) + run_out(NC) - 1 produce output: 58 cells per run for NC = 2,
// 56 for NC = 3.
__host__ __device__ constexpr int run_left(int nc) { return nc + 1; }
__host__ __device__ constexpr int run_out(int nc) { return WAVE - 2 * (nc + 1); }

// Control block in device memory. Every sweep of a step derives the step's dt
// and its go/no-go decision from it, so a captured sequence of steps needs no
// host involvement and no separate time-step kernel, and closing a step needs
// no inter-block synchronisation:
//   * rec[0], rec[1] hold the two most recent step states; the one with the
//     larger step count is current.
//   * The first sweep of a step records the running step's count in `started`
//     (-1 when the step does not run).
//   * Block 0 of the step's final sweep writes the next step state into the
//     older record with plain stores. Every other sweep of the step reads the
//     newer record, which the final sweep never writes; the final sweep itself
//     reads the record whose count equals `started`. Once the final sweep has
//     completed, the new record is the newer one.
//   * The CFL speed of the state with step count n is reduced (atomic max of
//     the bit images of non-negative doubles) into xcd[.].speed[n & 1], one
//     cache line per XCD; the first sweep of step n clears slot (n + 1) & 1.
//   * Block 0 of the first sweep of step n turns those speeds into the step's
//     dt and stores it in dt_step[n & 1]; the sweeps that finish a stage read
//     that one value. Where the first sweep itself finishes a stage (1D), its
//     blocks derive dt from the speeds directly.
struct StepRec {
    double t;          // time of the state
    double dt;         // time step that produced it (0 for an initial state)
    long long nsteps;  // steps taken to reach it
    long long pad;
};

struct alignas(128) XcdSlot {
    unsigned long long speed[2];
};

struct Ctl {
    StepRec rec[2];
    long long started;      // step count of the step in flight, -1 if none
    double t_final;         // stop time of the current run
    double cfl;             // CFL number
    double fixed_dt;        // > 0: fixed time step
    long long step_limit;   // a step starts only while nsteps < step_limit
    long long run_start;    // step count when the current run was set up
    double run_t0;          // time when the current run was set up
    int err;                // 1: a stage produced rho <= 0, p <= 0 or NaN
    int pad;
    long long bad_cell;     // smallest cell index of such a failure
    double dt_step[2];      // dt of step n in slot n & 1
    double sums[8];         // conserved sums (reduction output)
    XcdSlot xcd[8];
};

// The current step state, as the host reads it.
inline const StepRec& current_rec(const Ctl& c) { return c.rec[0].nsteps > c.rec[1].nsteps ? c.rec[0] : c.rec[1]; }

// Tables of the adaptive-order GP interpolation (indicator kind 3): whole-stencil
// GP weights of radius 3 and 2 at x_{i+1/2}, rows v_i / sqrt(lambda_i) of
// K_7(sigma) and K_5(sigma), the constants N/2 log(2 pi) + 1/2 log det K_N(sigma)
// for N = 7, 5, 3, and gamma_HI. The 3-point sub-stencils use Tab::wp,
// Tab::P[0] (K_3(sigma)) and Tab::gp (the CWENO linear weights). The weights
// of x_{i-1/2} are these mirrored (the host checks the identity).
template <typename Real>
struct AoTab {
    Real w7p[7], w5p[5];
    Real P7[7][7], P5[5][5];
    Real c[3];
    Real ghi;
};

// Interpolation tables of x_{i+1/2}; those of x_{i-1/2} are their mirror
// images, w_{R-m, R-j} and gamma_{R-m} (the host checks the identity).
template <typename Real>
struct Tab {
    Real wp[4][4];   // w_m at x_* = +1/2, [m][j] (the GP-AO sub-stencils)
    Real gwp[4][4];  // gamma_m w_m at x_* = +1/2 (GP-WENO and the polynomial schemes)
    Real gp[4];      // gamma_m for x_* = +1/2
    Real P[4][4][4];  // [m][i][j]: beta_m = sum_i (P[m][i] . f_m)^2 (GP: rows v_i / sqrt(lambda_i)
                      // of K_m(sigma), the same for every m; WENO-JS: a factor of the
                      // Jiang-Shu quadratic form of sub-stencil m)
    Real Ps[4][2];    // GP rows of R = 2, 3 on mirrored sums / differences (GpTablesF64::Ps)
    AoTab<Real> ao;
};

template <typename Real>
struct SweepArgs {
    const double* U;    // stage input state (stencil data)
    const double* Un;   // state at the start of the step (RK base)
    double* dU;         // direction accumulator of the right-hand side
    double* Uout;       // stage output (last direction of an RK stage)
    Ctl* ctl;
    int n[3];           // cells per axis
    int nseg;           // runs of cells per pencil along the sweep axis
    long long ncell;
    double inv_dx;      // 1/dx along the sweep axis
    double inv_dx_all[3];
    double gamma;
    double inv_gm1;     // 1/(gamma - 1)
    int first;          // first direction: the accumulator starts at zero
    int stage;          // 0: right-hand side only; 1..3: SSP-RK3 stage
    int positivity;     // positivity fallback of the Riemann states
    int step_start;     // first sweep of a step: clears the next speed slot
    int bc[2];          // boundary kinds of the sweep axis (low, high side)
    Tab<Real> tab;
};

// One problem of a batched launch: its buffers and geometry for one launch of
// the step sequence, and its range of logical blocks.
struct ProbDesc {
    const double* U;
    const double* Un;
    double* dU;
    double* Uout;
    Ctl* ctl;
    int n[3];
    int nseg;
    long long ncell;
    double inv_dx;
    double inv_dx_all[3];
    double gamma;
    double inv_gm1;     // 1/(gamma - 1)
    int positivity;
    int bc[2];          // boundary kinds of the sweep axis (low, high side)
    unsigned nblk;      // logical blocks of this problem in the launch
    long long block0;   // its first logical block
};

// Work table of one batched launch (device memory, rewritten by the host with
// stream-ordered copies when the set of problems changes).
struct BatchDir {
    const ProbDesc* probs;         // descriptors of the group's problems for this launch
    const unsigned short* owner;   // problem index of every logical block
    long long nblocks;             // logical blocks of the launch
    long long pad;
};

template <typename Real>
struct BatchArgs {
    const BatchDir* dir;   // the launch's work table
    int first;
    int stage;
    int step_start;
    Tab<Real> tab;
};

struct BatchStatus {
    double t;
    double dt;
    long long nsteps;
    int err;
    int pad;
};

// Which sweep kernel to launch: direction, stencil radius, whether it finishes
// an RK stage (last direction of stages 1..3; otherwise it accumulates into
// dU), the smoothness-indicator kind (0: GP, Tab::P[0] serves every
// sub-stencil; 1: a factor per sub-stencil, Jiang-Shu, R = 1, 2; 2: GP on the
// data minus the centre cell's value, non-zero mean; 3: adaptive-order GP,
// R = 2, 3), whether the sweep axis has a non-periodic side (the kernel reads
// bc[]; the periodic-only kernels skip that logic and its registers), the
// number of flux-correction terms (2, or 3 for indicator kind 0), and whether
// it is the batched kernel (args is a BatchArgs, blocks its grid) or the
// single-problem one (args is a SweepArgs, the grid follows from it).
struct LaunchSel {
    int dir;
    int R;
    bool fin;
    int ik;
    bool bcg;
    int nc;
    bool batch;
};

// Launchers (defined in gpweno_kernels.hip).
hipError_t launch_sweep(int ndim, bool fp32, const LaunchSel& k, const void* args, long long blocks, hipStream_t s);
hipError_t launch_set_run(Ctl* ctl, double t_final, long long step_limit, hipStream_t s);
// Sets up a run of at most max_steps more steps (max_steps < 0: no limit) from
// the current step count, read on the device, so the host need not wait for it.
hipError_t launch_set_run_rel(Ctl* ctl, double t_final, long long max_steps, hipStream_t s);
long long sweep_blocks(int ndim, int dir, bool fp32, const int n[3], int nseg);
hipError_t launch_gather_status(Ctl* const* ctls, int nprob, BatchStatus* out, hipStream_t s);
hipError_t launch_set_time(Ctl* ctl, double t, long long nsteps, double cfl, double fixed_dt, hipStream_t s);
hipError_t launch_speed(int ndim, const double* U, long long ncell, const double inv_dx[3], double gamma, Ctl* ctl,
                        hipStream_t s);
hipError_t launch_sums(int nv, const double* U, long long ncell, double* partials, int npart, Ctl* ctl,
                       hipStream_t s);
hipError_t launch_poison(double* U, int nv, long long ncell, long long cell, hipStream_t s);
// Prepares one step of a state the context is not bound to: sets the time-step
// rule and the end of the run (no step limit) and clears the CFL-speed slots of
// the current step, for launch_speed to fill from that state.
hipError_t launch_step_prep(Ctl* ctl, double cfl, double fixed_dt, double t_final, hipStream_t s);

}  // namespace gpw

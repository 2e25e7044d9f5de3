// shw_kernels.h -- launch interface between the host runtime and the HIP
// kernels (plain C++ types only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shw_math.h"

namespace shw {

// One 1D instance as the kernels see it.
struct Inst1D {
    long long off;        // first double of the instance in the state buffer
    long long cell_off;   // first cell of the instance in per-cell arrays
    int n;                // cells
    int bc_lo, bc_hi;
    int pad;
    double dx;
};

// One 2D instance.
struct Inst2D {
    long long off;
    long long cell_off;
    int nx, ny;
    int bc[4];
    double dx, dy;
};

// Per-instance time-loop state kept on the device.
struct InstState {
    double t;             // simulated time
    long long steps;      // steps taken since creation
    int code;             // 0 ok, 1 non-physical state met
    int pad;
};

// Launch parameters of the batched 1D time loop.
struct Loop1D {
    const Inst1D *inst;
    int n_inst;
    const int *order;          // instance processing order (largest first)
    int *queue;                // work counter (zeroed by the launcher)
    double *state;             // caller's state buffer
    double *alt;               // ping-pong buffer of the same size
    const double *t_end;       // per instance end time (CFL mode)
    const double *dt_fixed;    // per instance fixed step (NULL: CFL mode)
    long long max_steps;       // per instance step limit for this launch
    InstState *ist;
    const uint8_t *flags;      // per cell gate flags (GATED mode)
};

hipError_t launch_loop1d(int eq, const Loop1D &L, const DevParams &P, int grid,
                         hipStream_t stream);
int loop1d_max_blocks(int eq);
hipError_t launch_dt1d(int eq, const Inst1D *inst, int n_inst, const double *state,
                       const DevParams &P, double *dt_out, hipStream_t stream);

} // namespace shw

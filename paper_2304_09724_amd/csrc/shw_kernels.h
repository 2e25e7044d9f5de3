// shw_kernels.h -- launch interface between the host runtime and the HIP
// kernels (plain C++ types only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shw_math.h"
#include "gate_math.h"

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
    long long face_off;        // positivity safeguard: first double of this instance's
                               // face records (x-faces [20][ny][nx+1], then y-faces
                               // [20][ny+1][nx])
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
    uint8_t *flags;            // per cell gate flags (read in GATED mode; LEARNED
                               // writes them at gate steps, reads them in between)
    const GateLane *gate;      // packed network (LEARNED mode)
    float gate_logit_min;      // cells with logit >= this take the full reconstruction
    int gate_every;            // LEARNED: evaluate the network every this many steps
    double share;              // cell-updates per workgroup if the launch's estimated work
                               // were spread evenly; > 0 turns on work-based wave priority
    double *faces;             // positivity safeguard (NULL: off): per instance, planes
                               // [2M][n+1] of each face's flux and value at t_{n+1},
                               // instance i at 2M (cell_off + i)
    uint8_t *trouble;          // safeguard: one byte per cell
};

// Launch parameters of one 2D step over a batch (all pointers device-side).
struct Step2D {
    const Inst2D *inst;
    int n_inst;
    const int *tile_off[2];    // per sweep direction: first tile of each instance (n_inst+1)
    // the running instances of the current step, rebuilt by compact2d_kernel
    // after each step's step sizes are known: their ids in order (act_inst),
    // per sweep direction the first tile of each in the running tiles'
    // numbering (act_off[DIR], act_n + 1 entries), their number (act_n[0])
    // and the running tiles per direction (act_n[1], act_n[2])
    int *act_inst;
    int *act_off[2];
    int *act_n;
    double *state;             // caller's state buffer
    double *alt;               // ping-pong buffer
    int *parity;               // per instance: 1 = current state is in alt
    double *dt;                // per instance step of the current step (0 = skip)
    int *last;                 // per instance: the step ends exactly at t_end
    const double *dt_fixed;    // per instance fixed step (fixed-step mode)
    const double *t_end;       // per instance end time (CFL mode)
    long long *steps_left;     // per instance step budget
    double *smax;              // per instance max of (|u|+c)/dx + (|v|+c)/dy
    int *bad;                  // per instance sticky non-physical flag
    int *active;               // instances still running after the last step
    InstState *ist;
    uint8_t *flags;            // per cell gate flags (read in GATED mode; in LEARNED
                               // mode written by the gate kernel at each step)
    const GateLane *gate;      // packed network (LEARNED mode)
    float gate_logit_min;      // cells with logit >= this take the full reconstruction
    double *faces;             // positivity safeguard (NULL: off): each face's averaged
                               // flux and its values at t_{n+1} at the four edge nodes
    uint8_t *trouble;          // safeguard: one byte per cell
    int *guard;                // safeguard: per instance, repaired in this step
};

int sweep2d_tiles(int n_sweep, int n_trans, int lines);
hipError_t launch_speed2d(int eq, const Step2D &S, const DevParams &P, int use_parity,
                          hipStream_t stream);
hipError_t launch_step2d(int eq, const Step2D &S, const DevParams &P, int fixed,
                         const int total_tiles[2], int lines, hipStream_t stream);
hipError_t launch_settle2d(const Step2D &S, int m, hipStream_t stream);

hipError_t launch_gate_data1d(const Inst1D *inst, int n_inst, int max_n, const double *state,
                              const DevParams &P, double level, float *feat, uint8_t *label,
                              hipStream_t stream);
hipError_t launch_mlp_logits(const float *X, int n, const GateLane *G, float *logits,
                             hipStream_t stream);
hipError_t launch_mlp_grad(const float *X, const float *y, int n, const float *p, float pos_w,
                           float *grad, float *loss, hipStream_t stream);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int t, float lr,
                       hipStream_t stream);

hipError_t launch_loop1d(int eq, const Loop1D &L, const DevParams &P, int grid, int variant,
                         hipStream_t stream);
int loop1d_max_blocks(int eq, int variant, bool learned, bool guard);
hipError_t launch_dt1d(int eq, const Inst1D *inst, int n_inst, const double *state,
                       const DevParams &P, double *dt_out, hipStream_t stream);

} // namespace shw

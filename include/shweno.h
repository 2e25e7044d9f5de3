/*
 * shweno.h -- C ABI of the MI355X (gfx950) ADER-SHWENO library.
 *
 * The library advances one or many independent problems
 *     W_t + F(W)_x (+ G(W)_y) = 0,   W(x, 0) = W0(x)
 * on uniform Cartesian meshes with the one-stage ADER-SHWENO scheme of Luo,
 * Li, Qiu, Zhu and Chen (arXiv 2304.09724): the problem statement is sec. 2
 * eq. (1) and sec. 3 eq. (2); the state carried from step to step is the cell
 * averages W and the cell averages of the derivatives V = avg W_x (sec. 2.4,
 * eq. (vv)) and, in 2D, Y = avg W_y and Z = avg W_xy (sec. 3.2); one step is
 * the algorithm of sec. 4 (Steps 1-5).
 *
 * Conventions shared by every entry point
 *  - Every function returns a shw_status; nothing throws across the ABI.
 *  - Argument errors return SHW_EINVAL before any device work is queued.
 *  - Device memory for the state and the workspace is owned by the caller
 *    (allocated by any means, e.g. PyTorch); the library never frees it.  The
 *    library owns only the context object and what it allocates itself for
 *    the learned gate.
 *  - All device work is queued on the HIP stream given at creation, in
 *    order; calls documented as "synchronising" wait for that stream.
 *  - One context per stream; calls on one context are not re-entrant.
 *  - Non-physical states (a non-finite value, rho <= 0 or p <= 0 in a cell
 *    average) are detected on the device, are sticky per instance, and are
 *    reported as SHW_ENONPHYS by the next synchronising call; that instance
 *    stops advancing, the others continue.  shw_status_detail names it.
 *
 * State layout (one instance): planes [q][m][ny][nx] of doubles, x fastest;
 * q = 0 W, 1 V, (2D:) 2 Y, 3 Z; m conservative components (rho, rho u
 * [, rho v], E) for Euler, one for scalar equations.  Derivative averages
 * are in physical units.  A batch is the instances' blocks back to back, in
 * the order of the mesh array.
 */
#ifndef SHWENO_H
#define SHWENO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SHW_OK = 0,
    SHW_EINVAL = -1,     /* invalid argument (nothing was queued) */
    SHW_ENOMEM = -2,     /* host allocation failed */
    SHW_EDEVICE = -3,    /* a HIP call failed */
    SHW_ENONPHYS = -4,   /* a non-physical state was detected */
    SHW_ESTATE = -5,     /* call made in the wrong state (e.g. gate not loaded) */
    SHW_ESCRATCH = -6    /* the batch exceeds the static scratch of shw_advance1d_static */
} shw_status;

enum { SHW_ADVECTION = 0, SHW_BURGERS = 1, SHW_EULER = 2 };
enum { SHW_BC_PERIODIC = 0, SHW_BC_TRANSMISSIVE = 1, SHW_BC_REFLECTIVE = 2 };
enum { SHW_W_NONLINEAR = 0, SHW_W_LINEAR = 1, SHW_W_GATED = 2, SHW_W_LEARNED = 3 };

/* Number of parameters of the learned gate's network (16-32-32-1):
 * W1[32][16], b1[32], W2[32][32], b2[32], w3[32], b3, in that order. */
#define SHW_GATE_NFEATURES 16
#define SHW_GATE_NPARAMS 1633

/* One uniform mesh (sec. 2: cells I_j of width dx; sec. 3: cells I_ij).
 * dim 1: nx cells on [x0, x1], ny must be 1.  dim 2: nx x ny cells.
 * bc: x-low, x-high, y-low, y-high (SHW_BC_*); the two ends of a periodic
 * direction must both be periodic.  1D needs nx >= 3, 2D nx, ny >= 3. */
typedef struct {
    int dim;
    int nx, ny;
    double x0, x1, y0, y1;
    int bc[4];
} shw_mesh;

/* Scheme parameters.  eq: SHW_*; gamma: ratio of specific heats (Euler,
 * sec. 5 uses 1.4); adv_a, adv_b: advection speeds; cfl: Courant number for
 * the device-computed step (sec. 5 uses 0.9); eps: regulariser of the
 * nonlinear weights; lin_w: linear weights of the big stencil and the two
 * small ones (sec. 2.3: 0.994, 0.003, 0.003); charwise: Euler only,
 * reconstruct characteristic fields; weights: SHW_W_* — NONLINEAR is the
 * paper's SHWENO (sec. 2.3), LINEAR uses the linear weights everywhere, GATED
 * takes per-cell flags from shw_set_flags, LEARNED (Euler) evaluates the
 * learned gate; gate_threshold (0 < t < 1): a cell whose gate score
 * sigmoid(logit) is >= t takes the full nonlinear reconstruction;
 * gate_every (LEARNED, 1..1024; 1D): the gate is evaluated at the first step
 * of each call and then every gate_every steps of an instance; s steps after
 * an evaluation a cell takes the nonlinear weights if any cell within 2s of
 * it was flagged then (the distance the data of a reconstruction can travel
 * in s steps).  In 2D the gate runs at every step.  LEARNED overwrites the
 * per-cell flags of SHW_W_GATED.  In GATED and LEARNED modes a wave of cells
 * takes the characteristic path if any of its cells needs the nonlinear
 * weights; its linear-weight cells then get the big quartic of their
 * characteristic fields, equal to the componentwise one up to rounding.
 * positivity (0 or 1; Euler, 1D and 2D): 0 is the paper's scheme, which has
 * no limiter; 1 adds a safeguard that is not in the paper: in a step that
 * leaves a non-physical average (non-finite, rho <= 0 or p <= 0), every face
 * (2D: x- and y-face) next to such a cell takes the first-order HLLE flux of
 * the two averages at t_n (Einfeldt's wave-speed bounds), its state at x/t =
 * 0 standing for the face value(s) at t_{n+1}; the cells on both sides of
 * those faces are updated again, so the step stays conservative, and only a
 * cell still non-physical then stops its instance.  Steps that need no
 * repair are unchanged bit for bit; the workspace grows by 48 bytes (1D) or
 * 320 bytes (2D) and 1 byte per cell. */
typedef struct {
    int eq;
    int charwise;
    int weights;
    double gamma;
    double adv_a, adv_b;
    double cfl;
    double eps;
    double lin_w[3];
    double gate_threshold;
    int gate_every;
    int positivity;
} shw_params;

typedef struct shw_ctx shw_ctx;

/* Number of doubles of one instance's state (q * m * nx * ny), 0 if the mesh
 * or parameters are invalid. */
size_t shw_state_doubles(const shw_mesh *mesh, const shw_params *params);

/* Bytes of device workspace shw_create needs for this batch, 0 if invalid
 * (meshes of different dimensions, Burgers outside 1D, the learned gate
 * for another equation than Euler, the positivity safeguard for another
 * equation than Euler, or an invalid mesh or parameter set). */
size_t shw_workspace_bytes(const shw_mesh *meshes, int n_inst, const shw_params *params);

/* Create a context for n_inst instances (all with the same dim and params).
 * d_state: device buffer of sum(shw_state_doubles) doubles, the current
 * state (caller-owned; it holds the current state after every call).
 * d_workspace: device buffer of shw_workspace_bytes bytes (caller-owned,
 * contents irrelevant).  hip_stream: a hipStream_t (NULL = default).  Times
 * start at 0.  Synchronising. */
shw_status shw_create(const shw_mesh *meshes, int n_inst, const shw_params *params,
                      double *d_state, void *d_workspace, void *hip_stream,
                      shw_ctx **out);

/* Release the context (never the caller's buffers).  Safe on NULL. */
void shw_destroy(shw_ctx *ctx);

/* Copy one instance's state in (set) or out (get), layout as above.
 * src/dst on the device if *_on_device is non-zero, else in host memory
 * (then the call is synchronising).  Setting a state clears that
 * instance's non-physical flag. */
shw_status shw_set_state(shw_ctx *ctx, int inst, const double *src, int src_on_device);
shw_status shw_get_state(shw_ctx *ctx, int inst, double *dst, int dst_on_device);

/* Per-instance simulated time and step count (host arrays of n_inst);
 * either pointer may be NULL.  Synchronising.  shw_set_time sets t. */
shw_status shw_get_time(shw_ctx *ctx, double *t, long long *steps);
shw_status shw_set_time(shw_ctx *ctx, const double *t);

/* Step size from the CFL condition for every instance (host array of
 * n_inst): 1D dt = cfl dx / max_j(|u|+c); 2D dt = cfl / max_ij((|u|+c)/dx +
 * (|v|+c)/dy); scalar equations use |a| (advection) or |W| (Burgers); the
 * maxima run over the cell averages at t_n.  The Courant number is the
 * paper's (sec. 5 takes 0.9 for every run); the paper does not write the
 * formula out, and these forms are a reading of it (in 2D the sum of the two
 * directions' rates).  An instance whose averages are non-physical gets
 * SHW_ENONPHYS.  Synchronising. */
shw_status shw_compute_dt(shw_ctx *ctx, double *dt);

/* One time step of every instance (the one-stage update of sec. 4, Steps
 * 1-5: reconstruction, GRP at the interface points, the time-integrated
 * fluxes of eq. (flux) / eq. (fx2d), and the update of the averages and the
 * derivative averages) with the given step sizes (host array of n_inst;
 * entries <= 0 leave that instance alone; a non-finite entry is SHW_EINVAL).
 * Asynchronous. */
shw_status shw_step(shw_ctx *ctx, const double *dt);

/* One time step of every instance (sec. 4, Steps 1-5) with the step size its
 * own averages give under the CFL condition, computed on the device (the
 * shw_compute_dt value, with no end time to clamp to): the same state as
 * shw_compute_dt followed by shw_step.  Instances stopped on a non-physical
 * state stay stopped.  Synchronising; SHW_ENONPHYS as shw_advance_to. */
shw_status shw_step_cfl(shw_ctx *ctx);

/* Advance every instance i to time T[i] (host array) with steps of sec. 4
 * whose sizes come from the CFL condition of shw_compute_dt, computed on the
 * device from each step's own averages; the last step of each instance is
 * clamped to end exactly at T[i] (a reading: the paper's runs of sec. 5 stop
 * at their end times without saying how the last step is taken).  At most
 * max_steps steps per instance in this call.  Writes the number of steps
 * taken by each instance to steps_out (host array, may be NULL).
 * Synchronising; returns SHW_ENONPHYS if any instance went non-physical. */
shw_status shw_advance_to(shw_ctx *ctx, const double *T, long long max_steps,
                          long long *steps_out);

/* Per-cell gate flags for SHW_W_GATED (one byte per cell, non-zero = full
 * nonlinear reconstruction, zero = linear weights), for instance inst, from
 * host memory.  Synchronising. */
shw_status shw_set_flags(shw_ctx *ctx, int inst, const uint8_t *flags);

/* The per-cell flags of instance inst as the last step used them (GATED:
 * those set; LEARNED: the gate's decisions, in 1D the stored ones before
 * the 2s widening) into host memory (nx * ny bytes).  Synchronising. */
shw_status shw_get_flags(shw_ctx *ctx, int inst, uint8_t *flags);

/* ---- learned troubled-cell gate (an addition to the paper's method) ------
 * A small network (16 -> 32 -> 32 -> 1, ReLU) scores each cell of an Euler
 * batch from 16 features of the data its reconstruction reads (sec. 2.3):
 * per conservative component the signed shape of the jumps of the averages
 * and of the neighbours' derivative averages, normalised by its size, and
 * that size; and u / (|u| + c).  Cells whose probability of needing the
 * nonlinear weights is below the threshold use the linear weights, the rest
 * the full SHWENO reconstruction.  In 2D (sec. 3.2) a cell is scored along x
 * and along y from its normal components (rho, m_n, E) with the same network
 * and takes the nonlinear weights in both stages of both sweeps if either
 * score reaches the threshold.  The network runs in BF16 on the matrix
 * cores with FP32 accumulation; the scheme itself stays FP64.  Parameters:
 * W1[32][16], b1[32], W2[32][32], b2[32], w3[32], b3, as FP32. */

/* Load network parameters (host array of SHW_GATE_NPARAMS floats) into the
 * context for SHW_W_LEARNED.  Synchronising. */
shw_status shw_gate_load(shw_ctx *ctx, const float *params);

/* Training data from the method itself, 1D Euler batches: for every cell of
 * the batch (instances back to back) its features (d_features, device,
 * [cells][16] floats; per component c = rho, m, E with dl, dr the jumps of
 * the averages, gm, gp = dx V of the left/right neighbour and
 * S = |dl| + |dr| + |gm| + |gp|: (dl, dr, gm, gp) / S (0 if S < 1e-30) and
 * log2(S^2 + 1e-12) / 32; last u / (|u| + c); FP32 from FP64 differences)
 * and its label (d_labels, device, one byte: 1 if the cell's characteristic
 * nonlinear reconstruction gives the big stencil less than level times its
 * linear weight in some field).  level in (0, 1], else SHW_EINVAL.
 * Asynchronous. */
shw_status shw_gate_data(shw_ctx *ctx, double level, float *d_features, uint8_t *d_labels);

/* Bytes of the packed (matrix-instruction layout) form of the network, and
 * the packing of host parameters into host memory. */
size_t shw_gate_packed_bytes(void);
shw_status shw_gate_pack(const float *params, void *packed);

/* Logits of n samples (d_X: device [n][16] floats) with the packed network
 * d_packed (device copy of shw_gate_pack's output) on the matrix cores.
 * Asynchronous on hip_stream. */
shw_status shw_mlp_logits(const float *d_X, int n, const void *d_packed, float *d_logits,
                          void *hip_stream);

/* Mean weighted binary cross-entropy of sigmoid(logit) over n samples
 * (labels d_y in {0,1}, positives weighted by pos_weight) and its gradient
 * with respect to the FP32 parameters d_params (device, SHW_GATE_NPARAMS):
 * d_grad and *d_loss are overwritten.  FP32 forward and backward on the
 * vector units.  Asynchronous. */
shw_status shw_mlp_grad(const float *d_X, const float *d_y, int n, const float *d_params,
                        float pos_weight, float *d_grad, float *d_loss, void *hip_stream);

/* One Adam step (beta 0.9/0.999, eps 1e-8) on d_params with moments d_m, d_v
 * (device, zero before step 1); step counts from 1.  Asynchronous. */
shw_status shw_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int step,
                        float lr, void *hip_stream);

/* 2D: shw_advance_to runs the steps in chunks of 8 on the device and, by
 * default, replays each full chunk as one HIP graph captured at the first
 * use (kernels only, no memory operations); enable = 0 launches the kernels
 * one by one instead.  Results are identical either way. */
shw_status shw_set_graphs(shw_ctx *ctx, int enable);

/* Tile variant of the kernels (results are identical for all of them):
 * 1D, the persistent workgroup that advances one instance has 128, 256 or
 * 512 threads (2, 4 or 8 waves sharing its 62-cell chunks) for variant 0, 1,
 * 2 (default 1); 2D, a sweep tile is 1, 2 or 4 lines of 60 cells (default
 * 2, i.e. 4 lines).  SHW_EINVAL for another value. */
shw_status shw_set_tile(shw_ctx *ctx, int variant);
shw_status shw_get_tile(shw_ctx *ctx, int *variant);

/* Autotuner: times `steps` CFL steps of every instance (no end time within
 * reach) for each tile variant, warm, on the context's own batch, keeps the
 * fastest (written to *best; per-variant milliseconds to ms[3], may be NULL)
 * and leaves state and times as they were.  In 1D a variant with more threads
 * per instance within 3 % of the fastest is kept instead: the timed steps
 * keep every instance busy, while a whole run ends on its longest instance,
 * which more threads finish sooner.  d_scratch: caller-owned device
 * buffer of sum(shw_state_doubles) doubles for the saved state.  Steps
 * 1..100000.  Synchronising. */
shw_status shw_autotune(shw_ctx *ctx, double *d_scratch, int steps, int *best, float *ms);

/* Per-instance status (host array of n_inst): SHW_OK, or SHW_ENONPHYS for an
 * instance that met a non-physical state and stopped.  Synchronising. */
shw_status shw_instance_status(shw_ctx *ctx, int *codes);

/* First failing instance and a message for the last error (any may be
 * NULL). */
shw_status shw_status_detail(shw_ctx *ctx, int *bad_instance, char *msg, size_t msg_len);

/* Library version string. */
const char *shw_version(void);

/* ---- an entry point that allocates nothing --------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * shw_advance1d_static: the batched 1D time loop of shw_create +
 * shw_advance_to + shw_destroy (the same kernels; the same states and step
 * counts bit for bit), with every device buffer beyond the caller's state
 * (the ping-pong copy of the state, the instance descriptors and time-loop
 * state, the work counter; with the positivity safeguard its face records
 * and per-cell flags) carved out of a static array the library keeps on each
 * GPU it runs on: SHW_STATIC_SCRATCH_BYTES per GPU, held until the process
 * ends.  The call allocates no device or host memory (no hipMalloc or
 * hipFree, no heap allocation).
 *   meshes, n_inst, params: as shw_create, 1D only, weights NONLINEAR or
 *     LINEAR (no per-cell flags, no learned gate); at most
 *     SHW_STATIC_MAX_INSTANCES instances;
 *   d_state: the caller's device state (layout as above), taken as the state
 *     at t = 0 of every instance and advanced in place;
 *   T: host array of end times; each instance takes CFL steps to T[i], the
 *     last one clamped (as shw_advance_to), at most max_steps of them;
 *   steps_out: host array of the steps taken per instance (may be NULL);
 *   hip_stream: the stream the work is queued on (NULL = default).
 * Returns SHW_ESCRATCH, before any device work, if the batch's buffers exceed
 * SHW_STATIC_SCRATCH_BYTES or n_inst exceeds SHW_STATIC_MAX_INSTANCES;
 * SHW_EINVAL for other invalid arguments; SHW_ENONPHYS if an instance met a
 * non-physical state (that instance stopped there, steps_out is written);
 * SHW_EDEVICE if a HIP call failed.  Synchronising.  Every call on a GPU
 * uses that GPU's one array and keeps no state from an earlier call: calls
 * that overlap on one GPU (other threads or streams) race and must be
 * serialised by the caller. */
#define SHW_STATIC_SCRATCH_BYTES (64u << 20)
#define SHW_STATIC_MAX_INSTANCES 4096
shw_status shw_advance1d_static(const shw_mesh *meshes, int n_inst, const shw_params *params,
                                double *d_state, const double *T, long long max_steps,
                                long long *steps_out, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif

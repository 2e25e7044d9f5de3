// sweep1d.hip -- the 1D ADER-SHWENO time loop for a batch of independent
// problems, as one persistent launch.
//
// Each workgroup takes whole instances from a work counter (largest first)
// and advances each to its end time on its own: CFL step size (block max
// reduction), one fused sweep per step, its own ping-pong buffer.  No grid-wide
// synchronisation exists, so instances with very different step counts do
// not wait for one another.
//
// One sweep (sec. 4, Steps 1-5) works on chunks of 64 lanes: lane l holds cell
// j = c0 + l - 1.  Every lane reconstructs its cell (Step 1, sec. 2.3) and
// keeps the jets at both cell edges; the jet at the right edge moves one lane
// up, so lane l meets the two sides of face j - 1/2 and solves its GRP
// (leading term, linearised derivative Riemann problems, Lax-Wendroff
// procedure: Steps 2-3, sec. 2.1) and the Gauss-Lobatto flux (Step 4,
// eq. (flux), Remark 2).  The face results move one lane down and lanes 1..62
// update their cells (Step 5, eq. (cons) and eqs. (derave), (tay1d)).  A
// chunk advances 62 cells; lanes 0 and 63 only feed their neighbours.
#include "lanes.h"
#include "shw_kernels.h"
#include "sweep1d_math.h"

namespace shw {

namespace {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int CHUNK = WAVE - 2;

template <int EQ>
__device__ __forceinline__ bool bad_state(const double *W, const DevParams &P)
{
    constexpr int M = NComp<EQ, 1>::M;
    bool bad = false;
#pragma unroll
    for (int c = 0; c < M; ++c) bad |= !isfinite(W[c]);
    if constexpr (EQ == EULER) {
        // p > 0  <=>  2 rho E > (rho u)^2 when rho > 0
        bad |= !(W[0] > 0.0) || !(2.0 * W[0] * W[2] - W[1] * W[1] > 0.0);
    }
    return bad;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

// One sweep of one instance: src -> dst with step dt; returns true if a new
// cell average of this thread is non-physical.
// cell whose gate decision stands for index q (outside the mesh: the
// periodic image, else the nearest end cell, which covers the mirror images
// of a reflective end within the same window)
__device__ __forceinline__ int flag_cell(int q, int n, int bc_lo, int bc_hi)
{
    if (q < 0) return bc_lo == BC_PERIODIC ? ((q % n) + n) % n : 0;
    if (q >= n) return bc_hi == BC_PERIODIC ? q % n : n - 1;
    return q;
}

template <int EQ, int NB, bool LRN, bool GUARD>
__device__ __forceinline__ bool sweep_instance(const Inst1D &d, const double *__restrict__ src,
                                               double *__restrict__ dst, double dt,
                                               const DevParams &P,
                                               const uint8_t *__restrict__ flags, int gate_since,
                                               double *spd_out, double *__restrict__ faces)
{
    constexpr int M = NComp<EQ, 1>::M;
    const int lane = threadIdx.x % WAVE;
    const int wave = threadIdx.x / WAVE;
    const int n = d.n;
    const int nchunk = (n + CHUNK - 1) / CHUNK;
    const double idx = 1.0 / d.dx, dt_dx = dt * idx;
    double js[5];
    jet_scales(idx, js);
    bool bad = false;
    double spd = 0.0;       // largest wave speed of the new averages of this lane
    for (int ch = wave; ch < nchunk; ch += NB / WAVE) {
        const int j = ch * CHUNK + lane - 1;       // this lane's cell, -1..n+61
        const bool live = j <= n;
        // lanes past the end read the last ghost cell and discard the result
        const int jl = live ? j : n;
        double Wm[M], Vm[M], W0[M], V0[M], Wp[M], Vp[M];
        int s0 = jl;
        if (ch * CHUNK - 2 >= 0 && ch * CHUNK + CHUNK + 1 <= n - 1) {
            // the whole chunk's stencil (cells 62 ch - 2 .. 62 ch + 63) is
            // inside the instance: the same for every lane of the wave
            load_inner<M>(src, n, jl, Wm, Vm, W0, V0, Wp, Vp);
        } else {
            load_cell<EQ, M>(src, n, jl - 1, d.bc_lo, d.bc_hi, Wm, Vm);
            s0 = load_cell<EQ, M>(src, n, jl, d.bc_lo, d.bc_hi, W0, V0);
            load_cell<EQ, M>(src, n, jl + 1, d.bc_lo, d.bc_hi, Wp, Vp);
        }
        bool full = P.weights == W_NONLINEAR;
        if (P.weights == W_GATED) full = flags[d.cell_off + s0] != 0;
        if constexpr (LRN) {
            // the decisions of the last gate pass (gate_pass, run at this
            // step or gate_since steps ago): s steps after it, a cell can need
            // the nonlinear weights only if a cell flagged then lies within 2s
            // cells (its reconstruction reads its neighbours, and each step
            // updates a cell from the reconstructions next to it); a ghost
            // cell stands for the cell it copies, window included
            const int reach = 2 * gate_since;
            const int home = flag_cell(jl, n, d.bc_lo, d.bc_hi);
            unsigned any = 0;
            for (int o = -reach; o <= reach; ++o)
                any |= flags[d.cell_off + flag_cell(home + o, n, d.bc_lo, d.bc_hi)];
            full = any != 0;
        }
        double lo[5][M], hi[5][M];
        // one reconstruction path per wave: characteristic if any lane needs
        // the nonlinear weights
        const bool charpath = __any(full);
        recon_cell<EQ, M>(Wm, W0, Wp, Vm, Vp, d.dx, full, charpath, P, lo, hi);
        // right-edge jet of the left neighbour
        double prev[5][M];
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int c = 0; c < M; ++c) prev[a][c] = from_lane_below(hi[a][c]);
        double Fh[M], We[M];
        if (lane >= 1 && j >= 0 && live) {
            face1d<EQ, M>(prev, lo, js, dt, P, Fh, We);
        } else {
#pragma unroll
            for (int c = 0; c < M; ++c) { Fh[c] = 0.0; We[c] = 0.0; }
        }
        if constexpr (GUARD) {
            if (lane >= 1 && (lane <= CHUNK || j == n) && j >= 0 && j <= n) {
                // the safeguard's record of face j - 1/2 (each face once:
                // lanes 1..62, and the last face of the instance from lane 63
                // when n is a multiple of 62)
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    faces[c * (n + 1) + j] = Fh[c];
                    faces[(M + c) * (n + 1) + j] = We[c];
                }
            }
        }
        double Fn[M], Wn[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            Fn[c] = from_lane_above(Fh[c]);
            Wn[c] = from_lane_above(We[c]);
        }
        if (lane >= 1 && lane <= CHUNK && j >= 0 && j < n) {
            double Wnew[M], Vnew[M];
            update1d<M>(W0, Fh, Fn, We, Wn, dt_dx, idx, Wnew, Vnew);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                dst[c * n + j] = Wnew[c];
                dst[(M + c) * n + j] = Vnew[c];
            }
            bad |= bad_state<EQ>(Wnew, P);
            spd = fmax(spd, wave_speed<EQ>(Wnew, P));
        }
    }
    // the next step's CFL speed, one value per wave (a0.. of spd_out)
    spd = wave_max(spd);
    if (lane == 0) spd_out[wave] = spd;
    return bad;
}

// The learned gate's pass over an instance (every gate_every steps): each
// wave evaluates the network for the 64 cells of a chunk (all lanes take part
// in the matrix instructions) and the owners store the decisions in the
// per-cell flags, which the sweeps then read.  A pass of its own keeps the
// network's registers out of the sweep's.
template <int NB>
__device__ void gate_pass(const Inst1D &d, const double *__restrict__ src, const DevParams &P,
                          uint8_t *__restrict__ flags, const u32x4 *gate, float gate_logit_min)
{
    constexpr int M = 3;
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int n = d.n;
    const int nchunk = (n + CHUNK - 1) / CHUNK;
    const GateLane G = gate_lane_lds(gate, lane);
    for (int ch = wave; ch < nchunk; ch += NB / WAVE) {
        const int j = ch * CHUNK + lane - 1;
        const int jl = j <= n ? j : n;
        double Wm[M], Vm[M], W0[M], V0[M], Wp[M], Vp[M];
        if (ch * CHUNK - 2 >= 0 && ch * CHUNK + CHUNK + 1 <= n - 1) {
            load_inner<M>(src, n, jl, Wm, Vm, W0, V0, Wp, Vp);
        } else {
            load_cell<EULER, M>(src, n, jl - 1, d.bc_lo, d.bc_hi, Wm, Vm);
            load_cell<EULER, M>(src, n, jl, d.bc_lo, d.bc_hi, W0, V0);
            load_cell<EULER, M>(src, n, jl + 1, d.bc_lo, d.bc_hi, Wp, Vp);
        }
        float f[GATE_NF];
        gate_features1d(Wm, W0, Wp, Vm, Vp, d.dx, P.gamma, f);
        const bool full = gate_wave_logit(f, G) >= gate_logit_min;
        if (lane >= 1 && lane <= CHUNK && j >= 0 && j < n) flags[d.cell_off + j] = (uint8_t)full;
    }
}

// Positivity safeguard (an addition to the paper's scheme, which has no
// limiter; on when the launch carries face records).  After a sweep that left
// a non-physical average, a cell is troubled when its new average is
// non-physical (the test written as p = (g-1)(E - m^2/(2 rho)) > 0, so the
// decision rounds as a plain evaluation of that formula does).  Every face
// next to a troubled cell takes the first-order HLLE flux of the two averages
// at t_n instead, its state at x/t = 0 standing for the face value at t_{n+1};
// the cells on both sides of such a face are updated again from the sweep's
// records of their other face, so the step stays conservative.  One round:
// a cell still non-physical fails the instance as before.  The wave speeds of
// all new averages are reduced again for the next step.  Returns true if a
// cell of this thread is still non-physical.
__device__ __forceinline__ bool troubled(const double W[3], const DevParams &P)
{
    if (!isfinite(W[0]) || !isfinite(W[1]) || !isfinite(W[2]) || !(W[0] > 0.0)) return true;
    const double ke = 0.5 * W[1] * W[1] / W[0];
    return !((P.gamma - 1.0) * (W[2] - ke) > 0.0);
}

template <int NB>
__device__ bool guard_instance(const Inst1D &d, const double *__restrict__ src,
                               double *__restrict__ dst, double dt, const DevParams &P,
                               const double *__restrict__ faces, uint8_t *__restrict__ trouble,
                               double *spd_out)
{
    constexpr int M = 3;
    const int n = d.n, nf = n + 1;
    for (int j = threadIdx.x; j < n; j += NB) {
        const double W[M] = {dst[j], dst[n + j], dst[2 * n + j]};
        trouble[j] = (uint8_t)troubled(W, P);
    }
    __syncthreads();
    const double idx = 1.0 / d.dx, dt_dx = dt * idx;
    bool bad = false;
    double spd = 0.0;
    for (int j = threadIdx.x; j < n; j += NB) {
        // the neighbours' indices; a ghost stands for the cell it copies
        const int jl = j > 0 ? j - 1 : (d.bc_lo == BC_PERIODIC ? n - 1 : 0);
        const int jr = j < n - 1 ? j + 1 : (d.bc_hi == BC_PERIODIC ? 0 : n - 1);
        const bool tj = trouble[j] != 0;
        const bool fl = tj || trouble[jl] != 0, fr = tj || trouble[jr] != 0;
        double W[M];
        if (fl || fr) {
            double W0[M], V0[M], Wx[M], Vx[M], FL[M], EL[M], FR[M], ER[M], Vn[M];
            load_cell<EULER, M>(src, n, j, d.bc_lo, d.bc_hi, W0, V0);
            if (fl) {
                load_cell<EULER, M>(src, n, j - 1, d.bc_lo, d.bc_hi, Wx, Vx);
                hlle_face<1>(Wx, W0, P, FL, EL);
            } else {
#pragma unroll
                for (int c = 0; c < M; ++c) { FL[c] = faces[c * nf + j]; EL[c] = faces[(M + c) * nf + j]; }
            }
            if (fr) {
                load_cell<EULER, M>(src, n, j + 1, d.bc_lo, d.bc_hi, Wx, Vx);
                hlle_face<1>(W0, Wx, P, FR, ER);
            } else {
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    FR[c] = faces[c * nf + j + 1];
                    ER[c] = faces[(M + c) * nf + j + 1];
                }
            }
            update1d<M>(W0, FL, FR, EL, ER, dt_dx, idx, W, Vn);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                dst[c * n + j] = W[c];
                dst[(M + c) * n + j] = Vn[c];
            }
        } else {
#pragma unroll
            for (int c = 0; c < M; ++c) W[c] = dst[c * n + j];
        }
        bad |= bad_state<EULER>(W, P);
        spd = fmax(spd, wave_speed<EULER>(W, P));
    }
    spd = wave_max(spd);
    if (threadIdx.x % WAVE == 0) spd_out[threadIdx.x / WAVE] = spd;
    return bad;
}

// LRN: the learned-gate instantiation (Euler only); the others carry no gate
// code, which keeps its matrix-core accumulators out of their register count.
// Two persistent workgroups share a compute unit, and each SIMD issues from
// its oldest ready wave first: left to that order, an instance that landed on
// the younger workgroup runs at a fraction of its speed for as long as the
// older one keeps finding work, and a heavy one then ends the launch late.
// Each step the waves take a priority from their instance's remaining work
// (cells x steps left) against the launch's even share per workgroup, so the
// instances likely to finish last are issued first.
__device__ inline void work_priority(double work, double share)
{
    const int p = work >= 0.5 * share ? 3 : work >= 0.25 * share ? 2 : work >= 0.125 * share ? 1 : 0;
    switch (__builtin_amdgcn_readfirstlane(p)) {
    case 3: __builtin_amdgcn_s_setprio(3); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    default: __builtin_amdgcn_s_setprio(0); break;
    }
}

// Occupancy: at least two waves per SIMD (at most 256 registers a lane), one
// wave alone cannot hide its FP64 latencies; the Euler instances fit a third
// (168 registers, a few of them spilled).
template <int EQ, int NB, bool LRN, bool GUARD>
__global__ void __launch_bounds__(NB) __attribute__((amdgpu_waves_per_eu(EQ == EULER ? 3 : 2)))
loop1d_kernel(Loop1D Lp, DevParams P)
{
    constexpr int M = NComp<EQ, 1>::M;
    __shared__ int s_item;
    // per-wave CFL speeds, double-buffered by step: a sweep writes the speeds
    // of the averages it produces into one half while the step size of the
    // running step was read from the other
    __shared__ double s_spd[2][NB / WAVE];
    // per-wave non-physical flags of the averages a sweep produced, buffered
    // the same way
    __shared__ int s_bad[2][NB / WAVE];
    __shared__ u32x4 s_gate[EQ == EULER ? GATE_LDS_WORDS : 1];
    const int tid = threadIdx.x;
    if constexpr (LRN) {
        // the packed network, shared by the waves, transposed for the LDS
        gate_to_lds(Lp.gate, s_gate, tid, NB);
        __syncthreads();
    }
    for (;;) {
        if (tid == 0) s_item = atomicAdd(Lp.queue, 1);
        __syncthreads();
        // the same word for every lane: a scalar, and so is what is indexed by it
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= Lp.n_inst) break;
        const int i = Lp.order[item];
        const Inst1D d = Lp.inst[i];
        InstState st = Lp.ist[i];
        if (st.code != 0) continue;
        const long long nd = 2LL * M * d.n;
        double *A = Lp.state + d.off;
        double *B = Lp.alt + d.off;
        const double T = Lp.t_end ? Lp.t_end[i] : 0.0;
        const double dt_fix = Lp.dt_fixed ? Lp.dt_fixed[i] : 0.0;
        long long k = 0;
        int code = 0;
        int gate_since = 0;
        int buf = 0;              // s_spd[buf]: speeds of the averages in A, once k > 0
        while (k < Lp.max_steps) {
            double dt;
            bool last = false;
            if (Lp.dt_fixed) {
                if (!(dt_fix > 0.0)) break;
                dt = dt_fix;
            } else {
                if (!(st.t < T)) break;
                if (k == 0) {
                    // first step of the launch: a pass over the averages at t_n
                    double smax = 0.0;
                    for (int j = tid; j < d.n; j += NB) {
                        double W[M];
#pragma unroll
                        for (int c = 0; c < M; ++c) W[c] = A[c * d.n + j];
                        smax = fmax(smax, wave_speed<EQ>(W, P));
                    }
                    smax = wave_max(smax);
                    if (tid % WAVE == 0) s_spd[buf][tid / WAVE] = smax;
                    __syncthreads();
                }
                // CFL step size: block max of the per-wave speeds
                double smax = s_spd[buf][0];
#pragma unroll
                for (int w = 1; w < NB / WAVE; ++w) smax = fmax(smax, s_spd[buf][w]);
                dt = P.cfl * d.dx / smax;
                if (dt >= T - st.t) { dt = T - st.t; last = true; }
                if (Lp.share > 0.0)
                    work_priority(d.n * fmin((double)(Lp.max_steps - k), ceil((T - st.t) / dt)),
                                  Lp.share);
            }
            // the gate runs at the first step of a launch and every gate_every
            // steps of the instance; steps are separated by block barriers, so
            // the decisions one wave stores are seen by the other waves
            gate_since = (k == 0 || (st.steps + k) % Lp.gate_every == 0) ? 0 : gate_since + 1;
            if constexpr (LRN) {
                if (gate_since == 0) {
                    gate_pass<NB>(d, A, P, Lp.flags, s_gate, Lp.gate_logit_min);
                    __syncthreads();        // every decision stored before the sweep reads them
                }
            }
            double *faces = GUARD ? Lp.faces + 2LL * M * (d.cell_off + i) : nullptr;
            const bool bad = sweep_instance<EQ, NB, LRN, GUARD>(d, A, B, dt, P, Lp.flags, gate_since,
                                                                s_spd[buf ^ 1], faces);
            // one full barrier (with workgroup fences) a step orders the speeds
            // and flags in LDS and the gate's stored decisions for the next step
            const bool wave_bad = __any(bad);
            if (tid % WAVE == 0) s_bad[buf ^ 1][tid / WAVE] = wave_bad;
            __syncthreads();
            int any_bad = 0;
#pragma unroll
            for (int w = 0; w < NB / WAVE; ++w) any_bad |= s_bad[buf ^ 1][w];
            if constexpr (GUARD) {
                if (any_bad) {
                    const bool still = guard_instance<NB>(d, A, B, dt, P, faces,
                                                          Lp.trouble + d.cell_off, s_spd[buf ^ 1]);
                    __syncthreads();
                    any_bad = __syncthreads_or(still);
                }
            }
            buf ^= 1;
            double *tmp = A; A = B; B = tmp;
            ++k;
            st.t = last ? T : st.t + dt;
            if (any_bad) { code = 1; break; }
        }
        // the current state must end in the caller's buffer
        if (k & 1) {
            double *dst = Lp.state + d.off;
            for (long long e = tid; e < nd; e += NB) dst[e] = A[e];
        }
        if (tid == 0) {
            st.steps += k;
            st.code = code;
            Lp.ist[i] = st;
        }
        __syncthreads();
    }
}

template <int EQ>
__global__ void __launch_bounds__(BLOCK) dt1d_kernel(const Inst1D *inst, const double *state,
                                                     DevParams P, double *dt_out)
{
    constexpr int M = NComp<EQ, 1>::M;
    __shared__ double s_red[BLOCK / WAVE];
    const Inst1D d = inst[blockIdx.x];
    const double *A = state + d.off;
    double smax = 0.0;
    bool bad = false;
    for (int j = threadIdx.x; j < d.n; j += BLOCK) {
        double W[M];
#pragma unroll
        for (int c = 0; c < M; ++c) W[c] = A[c * d.n + j];
        bad |= bad_state<EQ>(W, P);
        if (!bad) smax = fmax(smax, wave_speed<EQ>(W, P));
    }
    smax = wave_max(smax);
    if (threadIdx.x % WAVE == 0) s_red[threadIdx.x / WAVE] = smax;
    const int any_bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) {
        double m = s_red[0];
        for (int w = 1; w < BLOCK / WAVE; ++w) m = fmax(m, s_red[w]);
        dt_out[blockIdx.x] = any_bad ? -1.0 : P.cfl * d.dx / m;
    }
}

__global__ void zero_int_kernel(int *p) { *p = 0; }

} // namespace

// workgroup size of tile variant v: 2, 4 or 8 waves per instance
static int loop1d_threads(int v) { return v == 0 ? 128 : v == 2 ? 512 : 256; }

// The kernel instance for an equation and mode: the learned gate (Euler) and
// the positivity safeguard (Euler) are instances of their own, so the
// paper's scheme runs with neither one's code in its register budget.
template <int NB>
static const void *loop1d_fn(int eq, bool learned, bool guard)
{
    if (eq == EULER) {
        if (learned)
            return guard ? (const void *)loop1d_kernel<EULER, NB, true, true>
                         : (const void *)loop1d_kernel<EULER, NB, true, false>;
        return guard ? (const void *)loop1d_kernel<EULER, NB, false, true>
                     : (const void *)loop1d_kernel<EULER, NB, false, false>;
    }
    if (eq == BURG) return (const void *)loop1d_kernel<BURG, NB, false, false>;
    return (const void *)loop1d_kernel<ADV, NB, false, false>;
}

static const void *loop1d_fn(int eq, bool learned, bool guard, int nb)
{
    return nb == 128 ? loop1d_fn<128>(eq, learned, guard)
           : nb == 512 ? loop1d_fn<512>(eq, learned, guard) : loop1d_fn<256>(eq, learned, guard);
}

hipError_t launch_loop1d(int eq, const Loop1D &L, const DevParams &P, int grid, int variant,
                         hipStream_t stream)
{
    zero_int_kernel<<<1, 1, 0, stream>>>(L.queue);
    const int nb = loop1d_threads(variant);
    const bool guard = eq == EULER && L.faces != nullptr;
    Loop1D l = L;
    DevParams p = P;
    void *args[] = {&l, &p};
    return hipLaunchKernel(loop1d_fn(eq, P.weights == W_LEARNED, guard, nb), dim3(grid), dim3(nb),
                           args, 0, stream);
}

int loop1d_max_blocks(int eq, int variant, bool learned, bool guard)
{
    const int nb = loop1d_threads(variant);
    int per_cu = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, loop1d_fn(eq, learned, guard && eq == EULER, nb), nb, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus < 1) cus = 1;
    return per_cu * cus;
}

hipError_t launch_dt1d(int eq, const Inst1D *inst, int n_inst, const double *state,
                       const DevParams &P, double *dt_out, hipStream_t stream)
{
    if (eq == EULER) dt1d_kernel<EULER><<<n_inst, BLOCK, 0, stream>>>(inst, state, P, dt_out);
    else if (eq == BURG) dt1d_kernel<BURG><<<n_inst, BLOCK, 0, stream>>>(inst, state, P, dt_out);
    else dt1d_kernel<ADV><<<n_inst, BLOCK, 0, stream>>>(inst, state, P, dt_out);
    return hipGetLastError();
}

} // namespace shw

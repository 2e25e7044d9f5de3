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
#include "shw_kernels.h"

namespace shw {

namespace {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int CHUNK = WAVE - 2;

// data of cell j of a 1D instance (ghost cells by the boundary conditions:
// periodic wrap; transmissive copies the nearest average with a zero
// derivative average; reflective mirrors, odd quantities change sign)
template <int EQ, int M>
__device__ __forceinline__ int load_cell(const double *__restrict__ base, int n, int j,
                                         int bc_lo, int bc_hi, double W[M], double V[M])
{
    int s = j;
    int kind = -1;   // -1 interior, else the boundary condition in force
    if (j < 0 || j >= n) {
        kind = j < 0 ? bc_lo : bc_hi;
        if (kind == BC_PERIODIC) s = j < 0 ? j + n : j - n;
        else if (kind == BC_TRANSMISSIVE) s = j < 0 ? 0 : n - 1;
        else s = j < 0 ? -1 - j : 2 * n - 1 - j;
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
        W[c] = base[c * n + s];
        V[c] = base[(M + c) * n + s];
    }
    if (kind == BC_TRANSMISSIVE) {
#pragma unroll
        for (int c = 0; c < M; ++c) V[c] = 0.0;
    } else if (kind == BC_REFLECTIVE) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const bool odd = EQ == EULER && c == 1;
            if (odd) W[c] = -W[c]; else V[c] = -V[c];
        }
    }
    return s;
}

// Step 1: reconstruction of one cell; lo/hi receive d^a W/dx^a at the left
// and right edge, a = 0..4.
template <int EQ, int M>
__device__ __forceinline__ void recon_cell(const double Wm[M], const double W0[M],
                                           const double Wp[M], const double Vm[M],
                                           const double Vp[M], double dx, bool full,
                                           const DevParams &P, double lo[5][M],
                                           double hi[5][M])
{
    const double idx = 1.0 / dx;
    double sc[5];
    sc[0] = 1.0; sc[1] = idx; sc[2] = idx * idx; sc[3] = sc[2] * idx; sc[4] = sc[2] * sc[2];
    if constexpr (EQ == EULER) {
        if (full && P.charwise) {
            double R[M][M], L[M][M], lam[M];
            euler_eigen<1, 0>(W0, P.gamma, R, L, lam);
            double clo[M][5], chi[M][5];
#pragma unroll
            for (int s = 0; s < M; ++s) {
                double am = 0, a0 = 0, ap = 0, bm = 0, bp = 0;
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    am += L[s][c] * Wm[c];
                    a0 += L[s][c] * W0[c];
                    ap += L[s][c] * Wp[c];
                    bm += L[s][c] * Vm[c];
                    bp += L[s][c] * Vp[c];
                }
                double q[5], w[3];
                big_quartic(am, a0, ap, dx * bm, dx * bp, q);
                nonlinear_weights(q, am, a0, ap, P, w);
                combine(q, am, a0, ap, w, P);
                edge_derivs(q, clo[s], chi[s]);
            }
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    double l = 0.0, h = 0.0;
#pragma unroll
                    for (int s = 0; s < M; ++s) {
                        l += R[c][s] * clo[s][a];
                        h += R[c][s] * chi[s][a];
                    }
                    lo[a][c] = l * sc[a];
                    hi[a][c] = h * sc[a];
                }
            return;
        }
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
        double q[5], l5[5], h5[5];
        big_quartic(Wm[c], W0[c], Wp[c], dx * Vm[c], dx * Vp[c], q);
        if (full) {
            double w[3];
            nonlinear_weights(q, Wm[c], W0[c], Wp[c], P, w);
            combine(q, Wm[c], W0[c], Wp[c], w, P);
        }
        edge_derivs(q, l5, h5);
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            lo[a][c] = l5[a] * sc[a];
            hi[a][c] = h5[a] * sc[a];
        }
    }
}

// Lax-Wendroff procedure (sec. 2.1.2, eq. (ck)) as power series in (x, t):
// w[c][a][k] is the coefficient of x^a t^k; the PDE W_t = -F(W)_x gives
// (k+1) w[a][k+1] = -(a+1) F[a+1][k].  Time level by time level, every series
// coefficient of the fluxes is formed once (products by the Cauchy rule).
template <int EQ, int M>
__device__ __forceinline__ void ck1d(double w[M][5][5], const DevParams &P)
{
    if constexpr (EQ == ADV) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int a = 0; a + k < 4; ++a)
                w[0][a][k + 1] = -P.adv_a * (double)(a + 1) / (double)(k + 1) * w[0][a + 1][k];
    } else if constexpr (EQ == BURG) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int a = 0; a + k < 4; ++a) {
                // F = W^2/2 at (a+1, k)
                double s = 0.0;
#pragma unroll
                for (int b = 0; b <= a + 1; ++b)
#pragma unroll
                    for (int j = 0; j <= k; ++j) s += w[0][b][j] * w[0][a + 1 - b][k - j];
                w[0][a][k + 1] = -0.5 * (double)(a + 1) / (double)(k + 1) * s;
            }
    } else {
        const double gm1 = P.gamma - 1.0;
        double r[5][5], u[5][5], mu[5][5], p[5][5], ep[5][5], epu[5][5];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int a = 0; a + k <= 4; ++a) {
                if (a == 0 && k == 0) {
                    r[0][0] = 1.0 / w[0][0][0];
                } else {
                    double s = 0.0;
#pragma unroll
                    for (int b = 0; b <= a; ++b)
#pragma unroll
                        for (int j = 0; j <= k; ++j)
                            if (b + j > 0) s += w[0][b][j] * r[a - b][k - j];
                    r[a][k] = -s * r[0][0];
                }
                double su = 0.0;
#pragma unroll
                for (int b = 0; b <= a; ++b)
#pragma unroll
                    for (int j = 0; j <= k; ++j) su += w[1][b][j] * r[a - b][k - j];
                u[a][k] = su;
                double sm = 0.0;
#pragma unroll
                for (int b = 0; b <= a; ++b)
#pragma unroll
                    for (int j = 0; j <= k; ++j) sm += w[1][b][j] * u[a - b][k - j];
                mu[a][k] = sm;
                p[a][k] = gm1 * (w[2][a][k] - 0.5 * sm);
                ep[a][k] = w[2][a][k] + p[a][k];
                double se = 0.0;
#pragma unroll
                for (int b = 0; b <= a; ++b)
#pragma unroll
                    for (int j = 0; j <= k; ++j) se += ep[b][j] * u[a - b][k - j];
                epu[a][k] = se;
            }
#pragma unroll
            for (int a = 0; a + k < 4; ++a) {
                const double f = -(double)(a + 1) / (double)(k + 1);
                w[0][a][k + 1] = f * w[1][a + 1][k];
                w[1][a][k + 1] = f * (mu[a + 1][k] + p[a + 1][k]);
                w[2][a][k + 1] = f * epu[a + 1][k];
            }
        }
    }
}

// Steps 2-4 at one face: GRP from the two one-sided jets, then the flux of
// eq. (flux) with the 4-point Gauss-Lobatto rule in time and the interface
// state at t + dt (eq. (tay1d)).
template <int EQ, int M>
__device__ __forceinline__ void face1d(const double JL[5][M], const double JR[5][M],
                                       double dt, const DevParams &P, double Fh[M],
                                       double We[M])
{
    double w[M][5][5];
    // leading term (sec. 2.1.1) and the derivative Riemann problems (eq. (lineq))
    if constexpr (EQ == EULER) {
        double Ws[M], R[M][M], L[M][M], lam[M];
        hllc_state<1>(JL[0], JR[0], P.gamma, Ws);
        euler_eigen<1, 0>(Ws, P.gamma, R, L, lam);
        double scale = 0.0;
#pragma unroll
        for (int s = 0; s < M; ++s) scale = fmax(scale, fabs(lam[s]));
#pragma unroll
        for (int c = 0; c < M; ++c) w[c][0][0] = Ws[c];
        const double inv_fact[5] = {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0};
#pragma unroll
        for (int a = 1; a < 5; ++a) {
            double ch[M];
#pragma unroll
            for (int s = 0; s < M; ++s) {
                double l = 0.0, r = 0.0;
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    l += L[s][c] * JL[a][c];
                    r += L[s][c] * JR[a][c];
                }
                ch[s] = upwind(lam[s], scale, l, r);
            }
#pragma unroll
            for (int c = 0; c < M; ++c) {
                double d = 0.0;
#pragma unroll
                for (int s = 0; s < M; ++s) d += R[c][s] * ch[s];
                w[c][a][0] = d * inv_fact[a];
            }
        }
    } else {
        double lam;
        if constexpr (EQ == ADV) {
            lam = P.adv_a;
            w[0][0][0] = upwind(lam, fabs(lam), JL[0][0], JR[0][0]);
        } else {
            w[0][0][0] = burgers_state(JL[0][0], JR[0][0]);
            lam = w[0][0][0];
        }
        const double inv_fact[5] = {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0};
#pragma unroll
        for (int a = 1; a < 5; ++a)
            w[0][a][0] = upwind(lam, fabs(lam), JL[a][0], JR[a][0]) * inv_fact[a];
    }
    ck1d<EQ, M>(w, P);
    // Gauss-Lobatto in time over [t_n, t_n + dt]
    const double taus[4] = {0.0, (0.5 - LOB_H) * dt, (0.5 + LOB_H) * dt, dt};
    const double wts[4] = {LOB_W0, LOB_W1, LOB_W1, LOB_W0};
#pragma unroll
    for (int c = 0; c < M; ++c) Fh[c] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double tau = taus[q];
        double Wt[M], F[M];
#pragma unroll
        for (int c = 0; c < M; ++c)
            Wt[c] = w[c][0][0] + tau * (w[c][0][1] + tau * (w[c][0][2] + tau * (w[c][0][3] + tau * w[c][0][4])));
        phys_flux_x<EQ, 1>(Wt, P, F);
#pragma unroll
        for (int c = 0; c < M; ++c) Fh[c] += wts[q] * F[c];
        if (q == 3) {
#pragma unroll
            for (int c = 0; c < M; ++c) We[c] = Wt[c];
        }
    }
}

template <int EQ>
__device__ __forceinline__ double wave_speed(const double *W, const DevParams &P)
{
    if constexpr (EQ == ADV) return fabs(P.adv_a);
    else if constexpr (EQ == BURG) return fabs(W[0]);
    else {
        const double u = W[1] / W[0];
        const double p = (P.gamma - 1.0) * (W[2] - 0.5 * W[1] * u);
        return fabs(u) + sqrt(P.gamma * p / W[0]);
    }
}

template <int EQ>
__device__ __forceinline__ bool bad_state(const double *W, const DevParams &P)
{
    constexpr int M = NComp<EQ, 1>::M;
    bool bad = false;
#pragma unroll
    for (int c = 0; c < M; ++c) bad |= !isfinite(W[c]);
    if constexpr (EQ == EULER) {
        const double p = (P.gamma - 1.0) * (W[2] - 0.5 * W[1] * W[1] / W[0]);
        bad |= !(W[0] > 0.0) || !(p > 0.0);
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
template <int EQ>
__device__ __forceinline__ bool sweep_instance(const Inst1D &d, const double *__restrict__ src,
                                               double *__restrict__ dst, double dt,
                                               const DevParams &P,
                                               const uint8_t *__restrict__ flags)
{
    constexpr int M = NComp<EQ, 1>::M;
    const int lane = threadIdx.x % WAVE;
    const int wave = threadIdx.x / WAVE;
    const int n = d.n;
    const int nchunk = (n + CHUNK - 1) / CHUNK;
    bool bad = false;
    for (int ch = wave; ch < nchunk; ch += BLOCK / WAVE) {
        const int j = ch * CHUNK + lane - 1;       // this lane's cell, -1..n+61
        const bool live = j <= n;
        double lo[5][M], hi[5][M], W0[M];
        if (live) {
            double Wm[M], Vm[M], Wp[M], Vp[M], V0[M];
            load_cell<EQ, M>(src, n, j - 1, d.bc_lo, d.bc_hi, Wm, Vm);
            const int s0 = load_cell<EQ, M>(src, n, j, d.bc_lo, d.bc_hi, W0, V0);
            load_cell<EQ, M>(src, n, j + 1, d.bc_lo, d.bc_hi, Wp, Vp);
            bool full = P.weights == W_NONLINEAR;
            if (P.weights == W_GATED) full = flags[d.cell_off + s0] != 0;
            recon_cell<EQ, M>(Wm, W0, Wp, Vm, Vp, d.dx, full, P, lo, hi);
        } else {
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int c = 0; c < M; ++c) { lo[a][c] = 1.0; hi[a][c] = 1.0; }
#pragma unroll
            for (int c = 0; c < M; ++c) W0[c] = 1.0;
        }
        // right-edge jet of the left neighbour
        double prev[5][M];
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int c = 0; c < M; ++c) prev[a][c] = __shfl_up(hi[a][c], 1, WAVE);
        double Fh[M], We[M];
        if (lane >= 1 && j >= 0 && live) {
            face1d<EQ, M>(prev, lo, dt, P, Fh, We);
        } else {
#pragma unroll
            for (int c = 0; c < M; ++c) { Fh[c] = 0.0; We[c] = 0.0; }
        }
        double Fn[M], Wn[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            Fn[c] = __shfl_down(Fh[c], 1, WAVE);
            Wn[c] = __shfl_down(We[c], 1, WAVE);
        }
        if (lane >= 1 && lane <= CHUNK && j >= 0 && j < n) {
            const double r = dt / d.dx, idx = 1.0 / d.dx;
            double Wnew[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                Wnew[c] = W0[c] - r * (Fn[c] - Fh[c]);
                dst[c * n + j] = Wnew[c];
                dst[(M + c) * n + j] = (Wn[c] - We[c]) * idx;
            }
            bad |= bad_state<EQ>(Wnew, P);
        }
    }
    return bad;
}

template <int EQ>
__global__ void __launch_bounds__(BLOCK) loop1d_kernel(Loop1D Lp, DevParams P)
{
    constexpr int M = NComp<EQ, 1>::M;
    __shared__ int s_item;
    __shared__ double s_red[BLOCK / WAVE];
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(Lp.queue, 1);
        __syncthreads();
        const int item = s_item;
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
        while (k < Lp.max_steps) {
            double dt;
            bool last = false;
            if (Lp.dt_fixed) {
                if (!(dt_fix > 0.0)) break;
                dt = dt_fix;
            } else {
                if (!(st.t < T)) break;
                // CFL step size from the averages at t_n (block max reduction)
                double smax = 0.0;
                for (int j = tid; j < d.n; j += BLOCK) {
                    double W[M];
#pragma unroll
                    for (int c = 0; c < M; ++c) W[c] = A[c * d.n + j];
                    smax = fmax(smax, wave_speed<EQ>(W, P));
                }
                smax = wave_max(smax);
                if (tid % WAVE == 0) s_red[tid / WAVE] = smax;
                __syncthreads();
                smax = s_red[0];
#pragma unroll
                for (int w = 1; w < BLOCK / WAVE; ++w) smax = fmax(smax, s_red[w]);
                __syncthreads();
                dt = P.cfl * d.dx / smax;
                if (dt >= T - st.t) { dt = T - st.t; last = true; }
            }
            const bool bad = sweep_instance<EQ>(d, A, B, dt, P, Lp.flags);
            const int any_bad = __syncthreads_or(bad);
            double *tmp = A; A = B; B = tmp;
            ++k;
            st.t = last ? T : st.t + dt;
            if (any_bad) { code = 1; break; }
        }
        // the current state must end in the caller's buffer
        if (k & 1) {
            double *dst = Lp.state + d.off;
            for (long long e = tid; e < nd; e += BLOCK) dst[e] = A[e];
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

hipError_t launch_loop1d(int eq, const Loop1D &L, const DevParams &P, int grid,
                         hipStream_t stream)
{
    zero_int_kernel<<<1, 1, 0, stream>>>(L.queue);
    if (eq == EULER) loop1d_kernel<EULER><<<grid, BLOCK, 0, stream>>>(L, P);
    else if (eq == BURG) loop1d_kernel<BURG><<<grid, BLOCK, 0, stream>>>(L, P);
    else loop1d_kernel<ADV><<<grid, BLOCK, 0, stream>>>(L, P);
    return hipGetLastError();
}

int loop1d_max_blocks(int eq)
{
    int per_cu = 0;
    hipError_t e;
    if (eq == EULER) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, loop1d_kernel<EULER>, BLOCK, 0);
    else if (eq == BURG) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, loop1d_kernel<BURG>, BLOCK, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, loop1d_kernel<ADV>, BLOCK, 0);
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

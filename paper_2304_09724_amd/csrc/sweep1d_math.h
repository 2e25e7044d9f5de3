// sweep1d_math.h -- per-cell and per-face arithmetic of the 1D sweep
// (reconstruction, GRP, Gauss-Lobatto flux), templated on the real type.
#pragma once

#include "shw_math.h"

namespace shw {

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


// data of cells j-1, j, j+1 when all three lie inside the instance (no
// boundary condition in force)
template <int M>
__device__ __forceinline__ void load_inner(const double *__restrict__ base, int n, int j,
                                           double Wm[M], double Vm[M], double W0[M],
                                           double V0[M], double Wp[M], double Vp[M])
{
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const double *w = base + (long long)c * n + j, *v = base + (long long)(M + c) * n + j;
        Wm[c] = w[-1]; W0[c] = w[0]; Wp[c] = w[1];
        Vm[c] = v[-1]; V0[c] = v[0]; Vp[c] = v[1];
    }
}

// Step 1: reconstruction of one cell; lo/hi receive d^a W/dxi^a at the left
// and right edge, a = 0..4, in the cell's coordinate xi = (x - x_j)/dx (the
// face turns them into x-derivatives: the derivative Riemann problems are
// linear in the jets, so one per-instance factor per order serves both).
// full: nonlinear weights, else the linear ones (the big quartic alone).
// charpath (Euler, characteristic reconstruction on): work in
// characteristic fields; a cell with linear weights gets the
// same polynomial either way (the big quartic is linear in its data), up to
// rounding, so callers choose the path once for a whole wave and the cheap
// component-wise form serves waves without nonlinear cells.
template <int EQ, int M, class Re>
SHW_HD void recon_cell(const Re Wm[M], const Re W0[M], const Re Wp[M], const Re Vm[M],
                       const Re Vp[M], double dx, bool full, bool charpath,
                       const DevParams &P, Re lo[5][M], Re hi[5][M])
{
    if constexpr (EQ == EULER) {
        if (charpath && P.charwise) {
            Char1<Re> E;
            char_1d(W0, P.gamma, E);
            // Adding a constant to the three averages adds it to the big
            // quartic's and the combined polynomial's constant term and
            // changes no smoothness indicator or weight; so the fields are
            // reconstructed from the neighbours' differences to this cell's
            // average (its own field values then being zero), and the
            // average is added back to the components' constant term below.
            Re em[M], ep[M];
#pragma unroll
            for (int c = 0; c < M; ++c) { em[c] = Wm[c] - W0[c]; ep[c] = Wp[c] - W0[c]; }
            Re cm[M], cp[M], dm[M], dp[M];
            char1_L(E, em, cm);
            char1_L(E, ep, cp);
            char1_L(E, Vm, dm);
            char1_L(E, Vp, dp);
            Re cq[M][5];
#pragma unroll
            for (int s = 0; s < M; ++s) {
                big_quartic_centred(cm[s], cp[s], Re(dx * dm[s]), Re(dx * dp[s]), cq[s]);
                if (full) {
                    Re w[3];
                    nonlinear_weights_jumps(cq[s], -cm[s], cp[s], P, w);
                    Re k[3];
                    combine_factors(w, P, k);
                    combine_centred(cq[s], -cm[s], cp[s], k);
                }
            }
            // back to the components on the five coefficients (R is linear:
            // the same polynomial as mapping the ten edge jets), then the
            // edge derivatives of each component
            Re pq[M][5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const Re y[M] = {cq[0][k], cq[1][k], cq[2][k]};
                Re x[M];
                char1_R(E, y, x);
#pragma unroll
                for (int c = 0; c < M; ++c) pq[c][k] = x[c];
            }
#pragma unroll
            for (int c = 0; c < M; ++c) pq[c][0] += W0[c];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                Re l5[5], h5[5];
                edge_derivs(pq[c], l5, h5);
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    lo[a][c] = l5[a];
                    hi[a][c] = h5[a];
                }
            }
            return;
        }
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
        Re q[5], l5[5], h5[5];
        big_quartic(Wm[c], W0[c], Wp[c], Re(dx * Vm[c]), Re(dx * Vp[c]), q);
        if (full) {
            Re w[3];
            nonlinear_weights(q, Wm[c], W0[c], Wp[c], P, w);
            Re k[3];
            combine_factors(w, P, k);
            combine(q, Wm[c], W0[c], Wp[c], k);
        }
        edge_derivs(q, l5, h5);
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            lo[a][c] = l5[a];
            hi[a][c] = h5[a];
        }
    }
}

// Lax-Wendroff procedure (sec. 2.1.2, eq. (ck)) as power series in (x, t):
// w[c][a][k] is the coefficient of x^a t^k; the PDE W_t = -F(W)_x gives
// (k+1) w[a][k+1] = -(a+1) F[a+1][k].  Time level by time level, every series
// coefficient of the fluxes is formed once (products by the Cauchy rule).
template <int EQ, int M, class R>
SHW_HD void ck1d(R w[M][5][5], const DevParams &P)
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
                R s = 0.0;
#pragma unroll
                for (int b = 0; b <= a + 1; ++b)
#pragma unroll
                    for (int j = 0; j <= k; ++j) s += w[0][b][j] * w[0][a + 1 - b][k - j];
                w[0][a][k + 1] = -0.5 * (double)(a + 1) / (double)(k + 1) * s;
            }
    } else {
        const double gm1 = P.gamma - 1.0;
        // velocity by series division (rho u = m), no reciprocal series
        const R r00 = recip(w[0][0][0]);
        R u[5][5], mu[5][5], p[5][5], ep[5][5], epu[5][5];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int a = 0; a + k <= 4; ++a) {
                R su = w[1][a][k];
#pragma unroll
                for (int b = 0; b <= a; ++b)
#pragma unroll
                    for (int j = 0; j <= k; ++j)
                        if (b + j > 0) su -= w[0][b][j] * u[a - b][k - j];
                u[a][k] = su * r00;
                R sm = 0.0;
#pragma unroll
                for (int b = 0; b <= a; ++b)
#pragma unroll
                    for (int j = 0; j <= k; ++j) sm += w[1][b][j] * u[a - b][k - j];
                mu[a][k] = sm;
                p[a][k] = gm1 * (w[2][a][k] - 0.5 * sm);
                ep[a][k] = w[2][a][k] + p[a][k];
                R se = 0.0;
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

// Per-instance factors of face1d: js[a] = dx^-a / a!, turning the jets' xi-
// derivatives of order a into Taylor coefficients in x.
SHW_HD void jet_scales(double idx, double js[5])
{
    js[0] = 1.0;
    js[1] = idx;
    js[2] = 0.5 * idx * idx;
    js[3] = (1.0 / 6.0) * idx * idx * idx;
    js[4] = (1.0 / 24.0) * (idx * idx) * (idx * idx);
}

// Steps 2-4 at one face: GRP from the two one-sided jets (xi-derivatives of
// the cells on either side; js from jet_scales), then the flux of eq. (flux)
// with the 4-point Gauss-Lobatto rule in time and the interface state at
// t + dt (eq. (tay1d)).
template <int EQ, int M, class Re>
SHW_HD void face1d(const Re JL[5][M], const Re JR[5][M], const double js[5], double dt,
                   const DevParams &P, Re Fh[M], Re We[M])
{
    Re w[M][5][5];
    // leading term (sec. 2.1.1) and the derivative Riemann problems (eq. (lineq))
    if constexpr (EQ == EULER) {
        Re Ws[M];
        Char1<Re> E;
        hllc_state<1>(JL[0], JR[0], P.gamma, Ws);
        char_1d(Ws, P.gamma, E);
        const Re lam[M] = {E.u - E.c, E.u, E.u + E.c};
        const Re scale = fabs(E.u) + E.c;
        // each field's side, chosen once for the four derivative orders
        // (the right side's weight is 1 - wl)
        Re wl[M];
#pragma unroll
        for (int s = 0; s < M; ++s) {
            Re wr;
            upwind_weights(lam[s], scale, wl[s], wr);
        }
#pragma unroll
        for (int c = 0; c < M; ++c) w[c][0][0] = Ws[c];
#pragma unroll
        for (int a = 1; a < 5; ++a) {
            // solved on the jump: each field's weights sum to one, so
            // R (w_l L x_L + w_r L x_R) = x_R + R (w_l L (x_L - x_R)) as R L = I,
            // one projection instead of two
            Re dj[M], l[M], d[M];
#pragma unroll
            for (int c = 0; c < M; ++c) dj[c] = JL[a][c] - JR[a][c];
            char1_L(E, dj, l);
#pragma unroll
            for (int s = 0; s < M; ++s) l[s] = wl[s] * l[s];
            char1_R(E, l, d);
#pragma unroll
            for (int c = 0; c < M; ++c) w[c][a][0] = (JR[a][c] + d[c]) * js[a];
        }
    } else {
        Re lam;
        if constexpr (EQ == ADV) {
            lam = P.adv_a;
            w[0][0][0] = upwind(lam, Re(fabs(P.adv_a)), JL[0][0], JR[0][0]);
        } else {
            w[0][0][0] = burgers_state(JL[0][0], JR[0][0]);
            lam = w[0][0][0];
        }
#pragma unroll
        for (int a = 1; a < 5; ++a)
            w[0][a][0] = upwind(lam, fabs(lam), JL[a][0], JR[a][0]) * js[a];
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
        Re Wt[M], F[M];
        // at tau = 0 the series is its constant term (the same value: the
        // compiler may not drop the zero products itself, since 0 * x is not
        // zero for every x)
#pragma unroll
        for (int c = 0; c < M; ++c)
            Wt[c] = q == 0 ? w[c][0][0]
                           : w[c][0][0] + tau * (w[c][0][1] + tau * (w[c][0][2] + tau * (w[c][0][3] + tau * w[c][0][4])));
        phys_flux_x<EQ, 1>(Wt, P, F);
#pragma unroll
        for (int c = 0; c < M; ++c) Fh[c] += wts[q] * F[c];
        if (q == 3) {
#pragma unroll
            for (int c = 0; c < M; ++c) We[c] = Wt[c];
        }
    }
}


// Largest characteristic speed of a cell average (CFL condition).
template <int EQ, class R>
SHW_HD R wave_speed(const R *W, const DevParams &P)
{
    if constexpr (EQ == ADV) return R(fabs(P.adv_a));
    else if constexpr (EQ == BURG) return fabs(W[0]);
    else {
        const R ir = recip(W[0]);
        const R u = W[1] * ir;
        const R p = (P.gamma - 1.0) * (W[2] - 0.5 * W[1] * u);
        return fabs(u) + sqrt_fast(P.gamma * p * ir);
    }
}

// Step 5 for one cell: new average from the two face fluxes (eq. (cons)) and
// new derivative average from the two interface states at t + dt (eq. (derave)).
template <int M, class R>
SHW_HD void update1d(const R W0[M], const R FL[M], const R FR[M], const R WL[M],
                     const R WR[M], double dt_dx, double inv_dx, R Wn[M], R Vn[M])
{
#pragma unroll
    for (int c = 0; c < M; ++c) {
        Wn[c] = W0[c] - dt_dx * (FR[c] - FL[c]);
        Vn[c] = (WR[c] - WL[c]) * inv_dx;
    }
}

} // namespace shw

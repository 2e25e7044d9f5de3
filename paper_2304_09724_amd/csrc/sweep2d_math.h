// sweep2d_math.h -- per-cell and per-interface-point arithmetic of the 2D
// sweep (sec. 3), templated on the real type.
//
// Everything here works in the frame of the sweep: "s" is the sweep direction
// (the interface normal) and "t" the transverse one.  For the x-sweep that is
// (x, y); the y-sweep runs the same code on the state seen with x and y
// exchanged (V and Y swapped, the two momentum components swapped), which is
// the same scheme because the Euler equations are invariant under that map.
#pragma once

#include "shw_math.h"

namespace shw {

// Index of the pair (a, n), a + n <= 4, in a 15-slot jet: d^{a+n}/ds^a dt^n.
SHW_HD constexpr int jidx(int a, int n)
{
    // rows n = 0..4 hold 5, 4, 3, 2, 1 entries
    return (n == 0 ? 0 : n == 1 ? 5 : n == 2 ? 9 : n == 3 ? 12 : 14) + a;
}

// --------------------------------------------------------------------------
// Stage 1 (sec. 3.2, first step): reconstruction across the sweep, in the
// transverse direction, of the line averages {W, Y} and of {V, Z} of one cell
// from the cell and its two transverse neighbours ([0] below, [1] the cell,
// [2] above).  One weight set (from the {W, Y} data) serves both, as one set
// of weights serves the function and its derivatives (sec. 2.1.2).  Euler:
// characteristic fields of the transverse Jacobian at the cell's average.
// full: nonlinear weights, else the linear ones (the big quartics alone);
// charpath (a whole wave's choice): work in characteristic fields, which for
// linear weights gives the componentwise polynomials up to rounding.
// Output: polynomials in eta = (t - t_j)/dt of the cell's line average of W
// (PW) and of W_s (PV), per conservative component.
// --------------------------------------------------------------------------
// Promises a caller may make at compile time (both false: nothing
// promised).  CHAR (Euler): P.charwise is on; a wave with a nonlinear-weight
// cell then takes the characteristic path, so the componentwise path never
// meets such a cell and its weights compile away.  FULL with CHAR: every
// cell takes the nonlinear weights (charpath holds for every wave), and the
// componentwise path compiles away.  The run-time tests stay as they are
// (their outcome is then known; keeping them left the compiler's register
// allocation of the sweeps better than folding them).
template <int M, int EQ, bool CHAR = false, bool FULL = false, class Re>
SHW_HD void stage1(const Re W[3][M], const Re V[3][M], const Re Y[3][M], const Re Z[3][M],
                   double dT, bool full, bool charpath, const DevParams &P, Re PW[M][5],
                   Re PV[M][5])
{
    static_assert(!CHAR || EQ == EULER, "characteristic path: Euler only");
    if constexpr (EQ == EULER) {
        if (charpath && P.charwise) {
            // The transverse Jacobian's fields (those of euler_eigen<2, 1>)
            // in closed form: the x-direction fields of the state with its
            // two momenta swapped, applied to data with the momenta swapped
            // (un-swapping R's rows gives exactly euler_eigen<2, 1>'s columns,
            // scaling included).
            const Re Ws[M] = {W[1][0], W[1][2], W[1][1], W[1][3]};
            CharX<Re> E;
            char_x(Ws, P.gamma, E);
            Re pw[3][M], pv[3][M], py[2][M], pz[2][M];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const Re xw[M] = {W[l][0], W[l][2], W[l][1], W[l][3]};
                const Re xv[M] = {V[l][0], V[l][2], V[l][1], V[l][3]};
                char_L(E, xw, pw[l]);
                char_L(E, xv, pv[l]);
            }
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                const Re xy[M] = {Y[2 * l][0], Y[2 * l][2], Y[2 * l][1], Y[2 * l][3]};
                const Re xz[M] = {Z[2 * l][0], Z[2 * l][2], Z[2 * l][1], Z[2 * l][3]};
                char_L(E, xy, py[l]);
                char_L(E, xz, pz[l]);
            }
            Re cw[M][5], cv[M][5];
#pragma unroll
            for (int f = 0; f < M; ++f) {
                const Re aw[3] = {pw[0][f], pw[1][f], pw[2][f]};
                const Re av[3] = {pv[0][f], pv[1][f], pv[2][f]};
                const Re bw[2] = {dT * py[0][f], dT * py[1][f]};
                const Re bv[2] = {dT * pz[0][f], dT * pz[1][f]};
                big_quartic(aw[0], aw[1], aw[2], bw[0], bw[1], cw[f]);
                big_quartic(av[0], av[1], av[2], bv[0], bv[1], cv[f]);
                // every lane of a characteristic wave combines (no divergent
                // branch); a linear-weight cell takes the factors (1, 0, 0),
                // which leave the big quartic as it is
                Re w[3];
                nonlinear_weights(cw[f], aw[0], aw[1], aw[2], P, w);
                Re k[3];
                combine_factors(w, P, k);
                if (!full) { k[0] = 1.0; k[1] = 0.0; k[2] = 0.0; }
                combine(cw[f], aw[0], aw[1], aw[2], k);
                combine(cv[f], av[0], av[1], av[2], k);
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const Re yw[M] = {cw[0][k], cw[1][k], cw[2][k], cw[3][k]};
                const Re yv[M] = {cv[0][k], cv[1][k], cv[2][k], cv[3][k]};
                Re xw[M], xv[M];
                char_R(E, yw, xw);
                char_R(E, yv, xv);
                // momenta back to their places
                PW[0][k] = xw[0]; PW[1][k] = xw[2]; PW[2][k] = xw[1]; PW[3][k] = xw[3];
                PV[0][k] = xv[0]; PV[1][k] = xv[2]; PV[2][k] = xv[1]; PV[3][k] = xv[3];
            }
            return;
        }
    }
    if constexpr (!(CHAR && FULL)) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
            big_quartic(W[0][c], W[1][c], W[2][c], Re(dT * Y[0][c]), Re(dT * Y[2][c]), PW[c]);
            big_quartic(V[0][c], V[1][c], V[2][c], Re(dT * Z[0][c]), Re(dT * Z[2][c]), PV[c]);
            if (!CHAR && full) {
                Re w[3];
                nonlinear_weights(PW[c], W[0][c], W[1][c], W[2][c], P, w);
                Re k[3];
                combine_factors(w, P, k);
                combine(PW[c], W[0][c], W[1][c], W[2][c], k);
                combine(PV[c], V[0][c], V[1][c], V[2][c], k);
            }
        }
    }
}

// Coefficient of (eta' - eta)^n of a quartic about eta (its n-th derivative
// over n!), times scale: sum_k C(k, n) c_k eta^(k-n), n = 0..4.
template <class Re>
SHW_HD Re taylor_at(const Re c[5], double eta, int n, double scale)
{
    const double e2 = eta * eta, e3 = e2 * eta, e4 = e2 * e2;
    switch (n) {
    case 0: return (c[0] + eta * c[1] + e2 * c[2] + e3 * c[3] + e4 * c[4]) * scale;
    case 1: return (c[1] + (2.0 * eta) * c[2] + (3.0 * e2) * c[3] + (4.0 * e3) * c[4]) * scale;
    case 2: return (c[2] + (3.0 * eta) * c[3] + (6.0 * e2) * c[4]) * scale;
    case 3: return (c[3] + (4.0 * eta) * c[4]) * scale;
    default: return c[4] * scale;
    }
}

// --------------------------------------------------------------------------
// Stage 2 (sec. 3.2, second step), one transverse order n at one edge node:
// reconstruction along the sweep direction from the node values a[l] =
// d^n/dt^n of the line averages of W of cells l = -1, 0, +1 and b[l] = the
// same for W_s of cells -1, +1 (scaled by ds inside).  Weights come from the
// order-0 data (w, the combination factors of combine_factors, is filled
// when n == 0 and reused for n >= 1).  Euler:
// characteristic fields of the sweep Jacobian at the cell's average (L, R),
// when charpath (a whole wave's choice; L, R are not read otherwise); full
// selects nonlinear or linear weights as in stage 1.
// Writes d^{a+n}W/ds^a dt^n at s = -1/2 (lo[a]) and s = +1/2 (hi[a]), a <= 4 - n,
// times scs[a] (with the node values' own scaling: the kernel's make them
// Taylor coefficients).
// --------------------------------------------------------------------------
template <int M, int EQ, bool CHAR = false, bool FULL = false, class Re>
SHW_HD void stage2_order(int n, const Re am[M], const Re a0[M], const Re ap[M], const Re bm[M],
                         const Re bp[M], const CharX<Re> &E, double dS,
                         const double scs[5], bool full, bool charpath, const DevParams &P,
                         Re w[M][3], Re lo[5][M], Re hi[5][M])
{
    static_assert(!CHAR || EQ == EULER, "characteristic path: Euler only");
    const bool proj = EQ == EULER && charpath && P.charwise;
    Re cq[M][5];
    bool done = false;
    if constexpr (EQ == EULER) {
        if (proj) {
            // Characteristic fields, centred as in 1D: the reconstruction
            // commutes with adding a constant to the three values, so the
            // fields of the neighbours' differences to this cell's value are
            // reconstructed and the value is added back to the components'
            // constant coefficient after R.
            Re em[M], ep[M], cm[M], cp[M], dm[M], dp[M];
#pragma unroll
            for (int c = 0; c < M; ++c) { em[c] = am[c] - a0[c]; ep[c] = ap[c] - a0[c]; }
            char_L(E, em, cm);
            char_L(E, ep, cp);
            char_L(E, bm, dm);
            char_L(E, bp, dp);
#pragma unroll
            for (int f = 0; f < M; ++f) {
                big_quartic_centred(cm[f], cp[f], Re(dS * dm[f]), Re(dS * dp[f]), cq[f]);
                // as in stage 1: every lane combines, a linear-weight cell
                // with the factors (1, 0, 0)
                if (n == 0) {
                    Re wn[3];
                    nonlinear_weights_jumps(cq[f], -cm[f], cp[f], P, wn);
                    combine_factors(wn, P, w[f]);
                    if (!full) { w[f][0] = 1.0; w[f][1] = 0.0; w[f][2] = 0.0; }
                }
                combine_centred(cq[f], -cm[f], cp[f], w[f]);
            }
            // back to the components on the five coefficients (R is linear:
            // the same polynomials as mapping the 2 (5 - n) edge jets)
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                Re y[M], x[M];
#pragma unroll
                for (int f = 0; f < M; ++f) y[f] = cq[f][k];
                char_R(E, y, x);
#pragma unroll
                for (int c = 0; c < M; ++c) cq[c][k] = x[c];
            }
#pragma unroll
            for (int c = 0; c < M; ++c) cq[c][0] += a0[c];
            done = true;
        }
    }
    if constexpr (!(CHAR && FULL)) {
        if (!done) {
#pragma unroll
            for (int c = 0; c < M; ++c) {
                big_quartic(am[c], a0[c], ap[c], Re(dS * bm[c]), Re(dS * bp[c]), cq[c]);
                if (!CHAR && full) {
                    if (n == 0) {
                        Re wn[3];
                        nonlinear_weights(cq[c], am[c], a0[c], ap[c], P, wn);
                        combine_factors(wn, P, w[c]);
                    }
                    combine(cq[c], am[c], a0[c], ap[c], w[c]);
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
        Re l5[5], h5[5];
        edge_derivs(cq[c], l5, h5);
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            if (a + n > 4) continue;
            lo[a][c] = l5[a] * scs[a];
            hi[a][c] = h5[a] * scs[a];
        }
    }
}

// --------------------------------------------------------------------------
// Lax-Wendroff procedure in two space dimensions (sec. 3.1), Euler: the
// conservative spatial series of the interface state (seeds s[c][a][b],
// coefficient of s^a t^b, a+b <= 4) is carried to its time layers.  The
// recursion runs on the primitive variables rho, u, v, p, whose PDE
// (rho_t = -(u rho_s + v rho_t' + rho (u_s + v_t')),
//  u_t = -(u u_s + v u_t' + p_s/rho), v_t likewise, p_t = -(u p_s + v p_t' +
//  g p (u_s + v_t'))) keeps fewer series alive (the divergence u_s + v_t'
// is formed once for the density and the pressure); the resulting conservative
// Taylor coefficients are the same numbers (the truncated series of one
// analytic solution), so only the rounding differs from a conservative-form
// recursion.  Output: the conservative time coefficients wt[c][k] at the
// interface point, k = 0..4, i.e. W(tau) = sum_k wt[k] tau^k.
//   spatial layer: rho = s0; u, v by series division of the momenta by rho;
//     p = (g-1)(E - (m_s u + m_t v)/2); r = 1/rho by series reciprocal;
//   level k -> k+1, each coefficient (a,b,k+1) from the Cauchy products of
//     the level <= k coefficients, divided by -(k+1);
//   back to conservative: m = rho u, E = p/(g-1) + (m_s u + m_t v)/2 along
//     the time line (a = b = 0).
// --------------------------------------------------------------------------
// The recursion itself is written out as straight-line code by gen_ck2d.py
// (one named scalar per series coefficient, so it stays in registers).
} // namespace shw
#include "ck2d_gen.h"
namespace shw {

// Linear advection W_t + a W_s + b W_t' = 0 (the same recursion, linear).
template <class R>
SHW_HD void ck2d_adv(const R s[5][5], double as, double at, R wt[5])
{
    R w[5][5][5];
#pragma unroll
    for (int a = 0; a <= 4; ++a)
#pragma unroll
        for (int b = 0; a + b <= 4; ++b) w[a][b][0] = s[a][b];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int a = 0; a + k <= 3; ++a)
#pragma unroll
            for (int b = 0; a + b + k <= 3; ++b)
                w[a][b][k + 1] = (-as * (double)(a + 1) / (double)(k + 1)) * w[a + 1][b][k]
                               + (-at * (double)(b + 1) / (double)(k + 1)) * w[a][b + 1][k];
#pragma unroll
    for (int k = 0; k <= 4; ++k) wt[k] = w[0][0][k];
}

// --------------------------------------------------------------------------
// GRP at one interface point with normal s (eqs. (taylor2d), (leadingterm2d),
// (lineq2d)).  grp2d_leading: the leading term from the two order-0 states
// (HLLC for Euler, upwind for advection) and the eigen-decomposition of the
// sweep Jacobian there.  grp2d_seed: one derivative d^{a+n}/ds^a dt^n
// (1 <= a+n <= 4) by upwinding each characteristic field between the cell
// below (JL, its s = +1/2 side) and above (JR); linear in the jets, so
// jets given as series coefficients (derivative / (a! n!)) give the
// series coefficient.
// --------------------------------------------------------------------------
template <int M, int EQ, class Re>
struct Leading2D {
    Re Ws[M], scale;
    CharX<Re> E;     // Euler: characteristic fields at Ws (speeds u-c, u, u, u+c)
    Re wl[M];        // Euler: each field's upwind weight of the left side (the
                     // right one is 1 - wl), shared by the 14 seeds
    Re lam0;         // advection: the speed
};

template <int M, int EQ, class Re>
SHW_HD void grp2d_leading(const Re JL[M], const Re JR[M], const DevParams &P, double as,
                          Leading2D<M, EQ, Re> &G)
{
    if constexpr (EQ == EULER) {
        hllc_state<2>(JL, JR, P.gamma, G.Ws);
        char_x(G.Ws, P.gamma, G.E);
        G.scale = fabs(G.E.u) + G.E.c;
        const Re lam[M] = {G.E.u - G.E.c, G.E.u, G.E.u, G.E.u + G.E.c};
#pragma unroll
        for (int f = 0; f < M; ++f) {
            Re wr;
            upwind_weights(lam[f], G.scale, G.wl[f], wr);
        }
    } else {
        G.lam0 = as;
        G.scale = fabs(as);
        G.Ws[0] = upwind(G.lam0, G.scale, JL[0], JR[0]);
    }
}

template <int M, int EQ, class Re>
SHW_HD void grp2d_seed(const Re JL[M], const Re JR[M], const Leading2D<M, EQ, Re> &G,
                       Re out[M])
{
    if constexpr (EQ == EULER) {
        // solved on the jump: each field's weights sum to one, so
        // R (w_l L x_L + w_r L x_R) = x_R + R (w_l L (x_L - x_R)) as R L = I,
        // one projection instead of two
        Re dj[M], l[M], d[M];
#pragma unroll
        for (int c = 0; c < M; ++c) dj[c] = JL[c] - JR[c];
        char_L(G.E, dj, l);
#pragma unroll
        for (int f = 0; f < M; ++f) l[f] = G.wl[f] * l[f];
        char_R(G.E, l, d);
#pragma unroll
        for (int c = 0; c < M; ++c) out[c] = JR[c] + d[c];
    } else {
        out[0] = upwind(G.lam0, G.scale, JL[0], JR[0]);
    }
}

// The whole GRP from full jets given as series coefficients
// (JL[jidx(a,n)][c] = d^{a+n}W/ds^a dt^n / (a! n!)): leading term, all
// derivatives, Lax-Wendroff; output time coefficients wt[c][k].
template <int M, int EQ, class Re>
SHW_HD void grp2d(const Re JL[15][M], const Re JR[15][M], const DevParams &P, double as,
                  double at, Re wt[M][5])
{
    Leading2D<M, EQ, Re> G;
    grp2d_leading<M, EQ>(JL[0], JR[0], P, as, G);
    Re s[M][5][5];
#pragma unroll
    for (int c = 0; c < M; ++c) s[c][0][0] = G.Ws[c];
#pragma unroll
    for (int n = 0; n <= 4; ++n)
#pragma unroll
        for (int a = 0; a + n <= 4; ++a) {
            if (a + n == 0) continue;
            Re o[M];
            grp2d_seed<M, EQ>(JL[jidx(a, n)], JR[jidx(a, n)], G, o);
#pragma unroll
            for (int c = 0; c < M; ++c) s[c][a][n] = o[c];
        }
    if constexpr (EQ == EULER) ck2d_euler(s, P.gamma, wt);
    else ck2d_adv(s[0], as, at, wt[0]);
}

// Flux of eq. (fx2d) at one edge node: 4-point Gauss-Lobatto in time of the
// s-flux of W(tau); also returns W(t + dt).
template <int M, int EQ, class Re>
SHW_HD void node_flux(const Re wt[M][5], double dt, const DevParams &P, double as, Re F[M],
                      Re We[M])
{
    const double taus[4] = {0.0, (0.5 - LOB_H) * dt, (0.5 + LOB_H) * dt, dt};
    const double wts[4] = {LOB_W0, LOB_W1, LOB_W1, LOB_W0};
#pragma unroll
    for (int c = 0; c < M; ++c) F[c] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double tau = taus[q];
        Re Wt[M], Fq[M];
        // at tau = 0 the series is its constant term (0 * x is not zero for
        // every x, so the compiler keeps the products otherwise)
#pragma unroll
        for (int c = 0; c < M; ++c)
            Wt[c] = q == 0 ? wt[c][0]
                           : wt[c][0] + tau * (wt[c][1] + tau * (wt[c][2] + tau * (wt[c][3] + tau * wt[c][4])));
        if constexpr (EQ == EULER) {
            phys_flux_x<EULER, 2>(Wt, P, Fq);
        } else {
            Fq[0] = as * Wt[0];
        }
#pragma unroll
        for (int c = 0; c < M; ++c) F[c] += wts[q] * Fq[c];
        if (q == 3) {
#pragma unroll
            for (int c = 0; c < M; ++c) We[c] = Wt[c];
        }
    }
}

} // namespace shw

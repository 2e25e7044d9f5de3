// shw_math.h -- device arithmetic of the ADER-SHWENO step for gfx950.
//
// Closed forms used by the sweep kernels.  Each function names the part of
// the paper (arXiv 2304.09724) it computes; the derivations are restated in
// the comments, so a reader can check them against the paper by hand.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

// Every arithmetic routine is a template on the real type R: the kernels use
// R = double; a host build with an operation-counting type measures the
// algorithmic flop count of exactly this code.
#define SHW_HD __host__ __device__ __forceinline__

namespace shw {

enum { ADV = 0, BURG = 1, EULER = 2 };
enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECTIVE = 2 };
enum { W_NONLINEAR = 0, W_LINEAR = 1, W_GATED = 2, W_LEARNED = 3 };

// Scheme parameters as the kernels see them.
struct DevParams {
    double gamma;
    double adv_a, adv_b;
    double cfl;
    double eps;
    double g1, g2, g3;   // linear weights: big quartic, left linear, right linear
    double inv_g1;       // 1 / g1
    int charwise;
    int weights;
};

// ---------------------------------------------------------------------------
// Reciprocals, quotients and square roots of the state arithmetic.  On the
// device in double precision they start from the hardware's approximate
// reciprocal (v_rcp_f64) or reciprocal square root (v_rsq_f64) and take two
// steps of Newton's iteration r <- r + r (1 - x r), or of Goldschmidt's
// iteration for sqrt(x) and 1/sqrt(x) together (g = x y, h = y/2;
// r = 1/2 - g h; g <- g + g r, h <- h + h r), each step squaring the relative
// error.  The results lie within about an ulp of the correctly rounded ones
// over the normal range (IEEE division and sqrt round to half an ulp but take
// twice the instructions).  A zero, negative, infinite or NaN argument gives
// a NaN or an infinity, as IEEE arithmetic gives a non-finite or a
// non-physical value there, so the step's checks still catch the state.
// Every other build (the host, the operation-counting type) uses IEEE
// division and sqrt, and counts one division or root per call.
// ---------------------------------------------------------------------------
template <class R>
SHW_HD R recip(R x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (std::is_same<R, double>::value) {
        double r = __builtin_amdgcn_rcp(x);
        double e = fma(-x, r, 1.0);
        r = fma(r, e, r);
        e = fma(-x, r, 1.0);
        return fma(r, e, r);
    }
#endif
    return 1.0 / x;
}

// a / b as a times the reciprocal of b (two roundings after the refinement).
template <class R>
SHW_HD R quot(R a, R b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (std::is_same<R, double>::value) return a * recip(b);
#endif
    return a / b;
}

// s = sqrt(x) and hs = 1/(2 sqrt(x)) (the iteration's own h).
template <class R>
SHW_HD void sqrt_hrsqrt(R x, R &s, R &hs)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (std::is_same<R, double>::value) {
        const double y = __builtin_amdgcn_rsq(x);
        double g = x * y, h = 0.5 * y;
        double r = fma(-g, h, 0.5);
        g = fma(g, r, g);
        h = fma(h, r, h);
        r = fma(-g, h, 0.5);
        g = fma(g, r, g);
        h = fma(h, r, h);
        s = g;
        hs = h;
        return;
    }
#endif
    s = sqrt(x);
    hs = 0.5 / s;
}


// sqrt(x) alone, from the same iteration (the reciprocal is not counted).
template <class R>
SHW_HD R sqrt_fast(R x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (std::is_same<R, double>::value) {
        double s, hs;
        sqrt_hrsqrt(x, s, hs);
        return s;
    }
#endif
    return sqrt(x);
}

template <int EQ, int DIM>
struct NComp { static constexpr int M = (EQ == EULER) ? (DIM == 1 ? 3 : 4) : 1; };

// 4-point Gauss-Lobatto on [-1/2, 1/2] (time rule of eq. (flux) per Remark 2,
// and the edge rule of eq. (fx2d)): nodes -1/2, -h, h, 1/2 with h = 1/(2 sqrt5),
// weights 1/12, 5/12, 5/12, 1/12.
constexpr double LOB_H = 0.22360679774997896964;
constexpr double LOB_W0 = 1.0 / 12.0;
constexpr double LOB_W1 = 5.0 / 12.0;

// ---------------------------------------------------------------------------
// SHWENO reconstruction of one scalar field on one cell (sec. 2.3).
// xi = (x - x_j)/dx.  Data: averages am, a0, ap of cells j-1, j, j+1 and the
// scaled derivative averages bm = dx V_{j-1}, bp = dx V_{j+1}.
// ---------------------------------------------------------------------------

// Quartic whose averages over cells -1, 0, 1 and whose increments
// p(l+1/2) - p(l-1/2) over cells -1, +1 match the data (solved by hand from
// those five linear conditions):
//   c0 = (1148 a0 - 94 s + 27 bd)/960, c1 = (13 d - 5 bs)/16,
//   c2 = (10 s - 20 a0 - 3 bd)/8, c3 = (bs - d)/4, c4 = (4 a0 - 2 s + bd)/4
// with s = am + ap, d = ap - am, bs = bm + bp, bd = bp - bm; each written as
// one sum of products with the divisions folded into the constants, so
// every term after the first is one FMA.
template <class R>
SHW_HD void big_quartic(R am, R a0, R ap, R bm, R bp, R c[5])
{
    const R s = am + ap, d = ap - am, bs = bm + bp, bd = bp - bm;
    c[0] = (1148.0 / 960.0) * a0 - (94.0 / 960.0) * s + (27.0 / 960.0) * bd;
    c[1] = 0.8125 * d - 0.3125 * bs;
    c[2] = 1.25 * s - 2.5 * a0 - 0.375 * bd;
    c[3] = 0.25 * bs - 0.25 * d;
    c[4] = a0 - 0.5 * s + 0.25 * bd;
}

// The same quartic for centred data (a0 = 0, am = cm, ap = cp).
template <class R>
SHW_HD void big_quartic_centred(R cm, R cp, R bm, R bp, R c[5])
{
    const R s = cm + cp, d = cp - cm, bs = bm + bp, bd = bp - bm;
    c[0] = (27.0 / 960.0) * bd - (94.0 / 960.0) * s;
    c[1] = 0.8125 * d - 0.3125 * bs;
    c[2] = 1.25 * s - 0.375 * bd;
    c[3] = 0.25 * bs - 0.25 * d;
    c[4] = 0.25 * bd - 0.5 * s;
}

// Nonlinear weights of the three candidates (big quartic, left linear a0 +
// (a0-am) xi, right linear a0 + (ap-a0) xi).  Smoothness indicators are
// sum_k int (d^k p/dxi^k)^2 over the cell; for the quartic that integral is
// the quadratic form below (exact integration of the squared derivatives).
// Simple-WENO weights: tau = ((|b1-b2| + |b1-b3|)/2)^2,
// w_l ~ g_l (1 + tau/(b_l + eps)).  The _jumps form takes dl = a0 - am and
// dr = ap - a0, all the averages enter through.
template <class R>
SHW_HD void nonlinear_weights_jumps(const R c[5], R dl, R dr, const DevParams &P, R w[3])
{
    const R b1 = c[1] * c[1] + 0.5 * c[1] * c[3] + (13.0 / 3.0) * c[2] * c[2]
                    + (21.0 / 5.0) * c[2] * c[4] + (3129.0 / 80.0) * c[3] * c[3]
                    + (87617.0 / 140.0) * c[4] * c[4];
    const R b2 = dl * dl, b3 = dr * dr;
    R tau = 0.5 * (fabs(b1 - b2) + fabs(b1 - b3));
    tau = tau * tau;
    // w_l = g_l (d_l + tau) / d_l with d_l = b_l + eps, normalised: over the
    // common denominator d1 d2 d3 a single division remains
    const R d1 = b1 + P.eps, d2 = b2 + P.eps, d3 = b3 + P.eps;
    const R w1 = P.g1 * (d1 + tau) * (d2 * d3);
    const R w2 = P.g2 * (d2 + tau) * (d1 * d3);
    const R w3 = P.g3 * (d3 + tau) * (d1 * d2);
    const R inv = recip(w1 + w2 + w3);
    w[0] = w1 * inv;
    w[1] = w2 * inv;
    w[2] = w3 * inv;
}

template <class R>
SHW_HD void nonlinear_weights(const R c[5], R am, R a0, R ap, const DevParams &P, R w[3])
{
    nonlinear_weights_jumps(c, a0 - am, ap - a0, P, w);
}

// Final polynomial (w1/g1)(p1 - g2 p2 - g3 p3) + w2 p2 + w3 p3 in place of the
// quartic coefficients c (the linear candidates only touch xi^0 and xi^1),
// written as f p1 + (w2 - f g2) p2 + (w3 - f g3) p3 with f = w1/g1:
// combine_factors forms k = (f, w2 - f g2, w3 - f g3) once per weight set,
// combine applies it to a quartic.
template <class R>
SHW_HD void combine_factors(const R w[3], const DevParams &P, R k[3])
{
    k[0] = w[0] * P.inv_g1;
    k[1] = w[1] - k[0] * P.g2;
    k[2] = w[2] - k[0] * P.g3;
}

template <class R>
SHW_HD void combine(R c[5], R am, R a0, R ap, const R k[3])
{
    const R dl = a0 - am, dr = ap - a0;
    c[0] = k[0] * c[0] + (k[1] + k[2]) * a0;
    c[1] = k[0] * c[1] + k[1] * dl + k[2] * dr;
    c[2] *= k[0];
    c[3] *= k[0];
    c[4] *= k[0];
}

// combine for centred data (a0 = 0, so the candidates' constant terms drop
// out): the same coefficients as combine(c, -dl, 0, dr, k).
template <class R>
SHW_HD void combine_centred(R c[5], R dl, R dr, const R k[3])
{
    c[0] *= k[0];
    c[1] = k[0] * c[1] + k[1] * dl + k[2] * dr;
    c[2] *= k[0];
    c[3] *= k[0];
    c[4] *= k[0];
}

// d^k p/dxi^k at xi = -1/2 (lo) and xi = +1/2 (hi), k = 0..4.
template <class R>
SHW_HD void edge_derivs(const R c[5], R lo[5], R hi[5])
{
    const R e0 = c[0] + 0.25 * c[2] + 0.0625 * c[4], o0 = 0.5 * c[1] + 0.125 * c[3];
    const R e1 = c[1] + 0.75 * c[3], o1 = c[2] + 0.5 * c[4];
    const R e2 = 2.0 * c[2] + 3.0 * c[4], o2 = 3.0 * c[3];
    const R e3 = 6.0 * c[3], o3 = 12.0 * c[4];
    hi[0] = e0 + o0; lo[0] = e0 - o0;
    hi[1] = e1 + o1; lo[1] = e1 - o1;
    hi[2] = e2 + o2; lo[2] = e2 - o2;
    hi[3] = e3 + o3; lo[3] = e3 - o3;
    hi[4] = 24.0 * c[4]; lo[4] = 24.0 * c[4];
}

// ---------------------------------------------------------------------------
// Euler equations (sec. 5, eqs. (Euler) and (2d)): E = p/(g-1) + rho|u|^2/2.
// ---------------------------------------------------------------------------

template <int DIM, class R>
SHW_HD R pressure(const R *W, double gamma)
{
    if constexpr (DIM == 1) {
        return (gamma - 1.0) * (W[2] - 0.5 * W[1] * W[1] / W[0]);
    } else {
        return (gamma - 1.0) * (W[3] - 0.5 * (W[1] * W[1] + W[2] * W[2]) / W[0]);
    }
}

// Eigenvectors of the flux Jacobian in direction DIR (0 = x, 1 = y) at W.
// R has the right eigenvectors as columns (speeds un-c, un, [un,] un+c), L =
// R^{-1} in closed form, with b1 = (g-1)/c^2 and b2 = b1 |u|^2 / 2.
template <int DIM, int DIR, class Re>
SHW_HD void euler_eigen(const Re *W, double gamma, Re R[][NComp<EULER, DIM>::M],
                        Re L[][NComp<EULER, DIM>::M], Re lam[NComp<EULER, DIM>::M])
{
    const Re ir = 1.0 / W[0];
    const Re u = W[1] * ir;
    if constexpr (DIM == 1) {
        const Re p = (gamma - 1.0) * (W[2] - 0.5 * W[1] * u);
        const Re c2 = gamma * p * ir;
        const Re c = sqrt(c2), ic = 1.0 / c;
        const Re H = (W[2] + p) * ir;
        const Re b1 = (gamma - 1.0) * (ic * ic), b2 = 0.5 * b1 * u * u;
        R[0][0] = 1.0;       R[0][1] = 1.0;         R[0][2] = 1.0;
        R[1][0] = u - c;     R[1][1] = u;           R[1][2] = u + c;
        R[2][0] = H - u * c; R[2][1] = 0.5 * u * u; R[2][2] = H + u * c;
        L[0][0] = 0.5 * (b2 + u * ic); L[0][1] = -0.5 * (b1 * u + ic); L[0][2] = 0.5 * b1;
        L[1][0] = 1.0 - b2;            L[1][1] = b1 * u;               L[1][2] = -b1;
        L[2][0] = 0.5 * (b2 - u * ic); L[2][1] = -0.5 * (b1 * u - ic); L[2][2] = 0.5 * b1;
        lam[0] = u - c; lam[1] = u; lam[2] = u + c;
    } else {
        const Re v = W[2] * ir;
        const Re q2 = u * u + v * v;
        const Re p = (gamma - 1.0) * (W[3] - 0.5 * W[0] * q2);
        const Re c2 = gamma * p * ir;
        const Re c = sqrt(c2), ic = 1.0 / c;
        const Re H = (W[3] + p) * ir;
        const Re b1 = (gamma - 1.0) * (ic * ic), b2 = 0.5 * b1 * q2;
        // normal (n) and tangential (s) velocity and momentum slots
        const Re un = DIR == 0 ? u : v, us = DIR == 0 ? v : u;
        constexpr int N = DIR == 0 ? 1 : 2, T = DIR == 0 ? 2 : 1;
        R[0][0] = 1.0; R[0][1] = 1.0; R[0][2] = 0.0; R[0][3] = 1.0;
        R[N][0] = un - c; R[N][1] = un; R[N][2] = 0.0; R[N][3] = un + c;
        R[T][0] = us; R[T][1] = us; R[T][2] = 1.0; R[T][3] = us;
        R[3][0] = H - un * c; R[3][1] = 0.5 * q2; R[3][2] = us; R[3][3] = H + un * c;
        L[0][0] = 0.5 * (b2 + un * ic); L[0][N] = -0.5 * (b1 * un + ic);
        L[0][T] = -0.5 * b1 * us;       L[0][3] = 0.5 * b1;
        L[1][0] = 1.0 - b2; L[1][N] = b1 * un; L[1][T] = b1 * us; L[1][3] = -b1;
        L[2][0] = -us; L[2][N] = 0.0; L[2][T] = 1.0; L[2][3] = 0.0;
        L[3][0] = 0.5 * (b2 - un * ic); L[3][N] = -0.5 * (b1 * un - ic);
        L[3][T] = -0.5 * b1 * us;       L[3][3] = 0.5 * b1;
        lam[0] = un - c; lam[1] = un; lam[2] = un; lam[3] = un + c;
    }
}

// The characteristic fields of the 1D Euler flux Jacobian at a state, held
// as the seven numbers its eigenvectors are built from instead of the 18
// entries of R and L (the matrices of euler_eigen<1, 0>): speeds u - c, u,
// u + c.  char1_L and char1_R apply L and R in closed form.  With b1 =
// (g-1)/c^2 and b2 = b1 u^2/2, L's coefficients are kept halved (hb1 = b1/2,
// hb2 = b2/2, hic = 1/(2c)): two of L's rows carry a factor 1/2, which then
// costs nothing, and halving is exact, so the rows' values are unchanged.
template <class Re>
struct Char1 {
    Re u, c, hic, H, hb1, hb2, hq;   // hq = u^2 / 2
};

template <class Re>
SHW_HD void char_1d(const Re *W, double gamma, Char1<Re> &E)
{
    const Re ir = recip(W[0]);
    E.u = W[1] * ir;
    E.hq = 0.5 * E.u * E.u;
    const Re p = (gamma - 1.0) * (W[2] - W[0] * E.hq);
    sqrt_hrsqrt(gamma * p * ir, E.c, E.hic);
    E.H = (W[2] + p) * ir;
    E.hb1 = (2.0 * (gamma - 1.0)) * (E.hic * E.hic);
    E.hb2 = E.hb1 * E.hq;
}

// y = L x: rows (b2 + u/c, -(b1 u + 1/c), b1)/2, (1 - b2, b1 u, -b1),
// (b2 - u/c, -(b1 u - 1/c), b1)/2; with s = b2 x0 - b1 (u x1 - x2) and
// d = (u x0 - x1)/c: y = ((s + d)/2, x0 - s, (s - d)/2), formed from s/2, d/2
template <class Re>
SHW_HD void char1_L(const Char1<Re> &E, const Re x[3], Re y[3])
{
    const Re hs = E.hb2 * x[0] - E.hb1 * (E.u * x[1] - x[2]);
    const Re hd = E.hic * (E.u * x[0] - x[1]);
    y[0] = hs + hd;
    y[1] = x[0] - 2.0 * hs;
    y[2] = hs - hd;
}

// x = R y: columns (1, u - c, H - u c), (1, u, u^2/2), (1, u + c, H + u c);
// with s = y0 + y1 + y2 and d = y2 - y0: x = (s, u s + c d,
// H s + (u^2/2 - H) y1 + u c d)
template <class Re>
SHW_HD void char1_R(const Char1<Re> &E, const Re y[3], Re x[3])
{
    const Re s = y[0] + y[1] + y[2], d = y[2] - y[0];
    x[0] = s;
    x[1] = E.u * s + E.c * d;
    x[2] = E.H * s + (E.hq - E.H) * y[1] + (E.u * E.c) * d;
}

// The characteristic fields of the 2D Euler flux Jacobian in x at a state,
// held as the eight numbers its eigenvectors are built from instead of the
// 32 entries of R and L (the same matrices as euler_eigen<2, 0>): speeds
// u - c, u, u, u + c.  char_L and char_R apply L and R in closed form.
template <class Re>
struct CharX {
    Re u, v, c, hic, H, hb1, hb2, hq;   // hq = |u|^2 / 2; halved as in Char1
};

template <class Re>
SHW_HD void char_x(const Re *W, double gamma, CharX<Re> &E)
{
    const Re ir = recip(W[0]);
    E.u = W[1] * ir;
    E.v = W[2] * ir;
    E.hq = 0.5 * (E.u * E.u + E.v * E.v);
    const Re p = (gamma - 1.0) * (W[3] - W[0] * E.hq);
    sqrt_hrsqrt(gamma * p * ir, E.c, E.hic);
    E.H = (W[3] + p) * ir;
    E.hb1 = (2.0 * (gamma - 1.0)) * (E.hic * E.hic);
    E.hb2 = E.hb1 * E.hq;
}

// y = L x: rows (b2 + u/c, -(b1 u + 1/c), -b1 v, b1)/2, (1 - b2, b1 u, b1 v,
// -b1), (-v, 0, 1, 0), (b2 - u/c, -(b1 u - 1/c), -b1 v, b1)/2; formed from the
// halves of s = b2 x0 - b1 (u x1 + v x2 - x3) and d = (u x0 - x1)/c as in char1_L
template <class Re>
SHW_HD void char_L(const CharX<Re> &E, const Re x[4], Re y[4])
{
    const Re hs = E.hb2 * x[0] - E.hb1 * (E.u * x[1] + E.v * x[2] - x[3]);
    const Re hd = E.hic * (E.u * x[0] - x[1]);
    y[0] = hs + hd;
    y[1] = x[0] - 2.0 * hs;
    y[2] = x[2] - E.v * x[0];
    y[3] = hs - hd;
}

// x = R y: columns (1, u - c, v, H - u c), (1, u, v, |u|^2/2), (0, 0, 1, v),
// (1, u + c, v, H + u c); with s = y0 + y1 + y3 and d = y3 - y0:
// x = (s, u s + c d, v s + y2, H s + (|u|^2/2 - H) y1 + u c d + v y2)
template <class Re>
SHW_HD void char_R(const CharX<Re> &E, const Re y[4], Re x[4])
{
    const Re s = y[0] + y[1] + y[3], d = y[3] - y[0];
    x[0] = s;
    x[1] = E.u * s + E.c * d;
    x[2] = E.v * s + y[2];
    x[3] = E.H * s + (E.hq - E.H) * y[1] + (E.u * E.c) * d + E.v * y[2];
}

// Physical flux in x of a point state (scalar equations: a W or W^2/2).
template <int EQ, int DIM, class R>
SHW_HD void phys_flux_x(const R *W, const DevParams &P, R *F)
{
    if constexpr (EQ == ADV) {
        F[0] = P.adv_a * W[0];
    } else if constexpr (EQ == BURG) {
        F[0] = 0.5 * W[0] * W[0];
    } else if constexpr (DIM == 1) {
        const R u = quot(W[1], W[0]);
        const R p = (P.gamma - 1.0) * (W[2] - 0.5 * W[1] * u);
        F[0] = W[1];
        F[1] = W[1] * u + p;
        F[2] = (W[2] + p) * u;
    } else {
        const R ir = recip(W[0]);
        const R u = W[1] * ir;
        const R p = (P.gamma - 1.0) * (W[3] - 0.5 * (W[1] * W[1] + W[2] * W[2]) * ir);
        F[0] = W[1];
        F[1] = W[1] * u + p;
        F[2] = W[2] * u;
        F[3] = (W[3] + p) * u;
    }
}

// HLLC Godunov state at x/t = 0 (leading term, sec. 2.1.1), Davis wave-speed
// estimates, contact speed from the HLLC jump conditions; a state on a
// boundary between two branches goes to the left one.
template <int DIM, class R>
SHW_HD void hllc_state(const R *WL, const R *WR, double gamma, R *Ws)
{
    constexpr int M = NComp<EULER, DIM>::M;
    const R rl = WL[0], rr = WR[0];
    const R irl = recip(rl), irr = recip(rr);
    const R ul = WL[1] * irl, ur = WR[1] * irr;
    R kl = WL[1] * ul, kr = WR[1] * ur;                   // rho |u|^2
    if constexpr (DIM == 2) {
        kl = kl + WL[2] * (WL[2] * irl);
        kr = kr + WR[2] * (WR[2] * irr);
    }
    const R pl = (gamma - 1.0) * (WL[M - 1] - 0.5 * kl);
    const R pr = (gamma - 1.0) * (WR[M - 1] - 0.5 * kr);
    const R cl = sqrt_fast(gamma * pl * irl), cr = sqrt_fast(gamma * pr * irr);
    const R SL = fmin(ul - cl, ur - cr);
    const R SR = fmax(ul + cl, ur + cr);
    const R ml = rl * (SL - ul), mr = rr * (SR - ur);
    const R Ss = quot(pr - pl + ul * ml - ur * mr, ml - mr);
    if (0.0 <= SL) {
#pragma unroll
        for (int c = 0; c < M; ++c) Ws[c] = WL[c];
        return;
    }
    if (0.0 > SR) {
#pragma unroll
        for (int c = 0; c < M; ++c) Ws[c] = WR[c];
        return;
    }
    const bool left = 0.0 <= Ss;
    const R *WK = left ? WL : WR;
    const R uk = left ? ul : ur, pk = left ? pl : pr;
    const R SK = left ? SL : SR, mk = left ? ml : mr;
    const R irk = left ? irl : irr;
    const R f = quot(mk, SK - Ss);
    Ws[0] = f;
    Ws[1] = f * Ss;
    if constexpr (DIM == 2) Ws[2] = f * (WK[2] * irk);
    Ws[M - 1] = f * (WK[M - 1] * irk + (Ss - uk) * (Ss + quot(pk, mk)));
}

// First-order HLLE flux F and state Ws at x/t = 0 in the normal direction x
// (the positivity safeguard's face, not part of the paper's scheme): a single
// intermediate state between wave-speed bounds after Einfeldt (1988), the
// smaller and larger of the sides' acoustic speeds and of the speeds of the
// Roe average (sqrt(rho) weights on u, v and the enthalpy).  With these bounds
// the first-order scheme keeps density and pressure positive.
template <int DIM, class R>
SHW_HD void hlle_face(const R *WL, const R *WR, const DevParams &P, R *F, R *Ws)
{
    constexpr int M = NComp<EULER, DIM>::M;
    const double g = P.gamma;
    const R irl = 1.0 / WL[0], irr = 1.0 / WR[0];
    const R ul = WL[1] * irl, ur = WR[1] * irr;
    R vl = 0.0, vr = 0.0;
    if constexpr (DIM == 2) { vl = WL[2] * irl; vr = WR[2] * irr; }
    const R pl = pressure<DIM>(WL, g), pr = pressure<DIM>(WR, g);
    const R sl = sqrt(WL[0]), sr = sqrt(WR[0]), iw = 1.0 / (sl + sr);
    const R ut = (sl * ul + sr * ur) * iw, vt = (sl * vl + sr * vr) * iw;
    const R ht = (sl * ((WL[M - 1] + pl) * irl) + sr * ((WR[M - 1] + pr) * irr)) * iw;
    const R ct = sqrt((g - 1.0) * (ht - 0.5 * (ut * ut + vt * vt)));
    const R SL = fmin(ul - sqrt(g * pl * irl), ut - ct);
    const R SR = fmax(ur + sqrt(g * pr * irr), ut + ct);
    R FL[M], FR[M];
    phys_flux_x<EULER, DIM>(WL, P, FL);
    phys_flux_x<EULER, DIM>(WR, P, FR);
    if (0.0 <= SL || SR <= 0.0) {
        const bool left = 0.0 <= SL;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            F[c] = left ? FL[c] : FR[c];
            Ws[c] = left ? WL[c] : WR[c];
        }
        return;
    }
    const R id = 1.0 / (SR - SL);
#pragma unroll
    for (int c = 0; c < M; ++c) {
        F[c] = (SR * FL[c] - SL * FR[c] + SL * SR * (WR[c] - WL[c])) * id;
        Ws[c] = (SR * WR[c] - SL * WL[c] - (FR[c] - FL[c])) * id;
    }
}

// Upwind solution at x/t = 0 of a linear Riemann problem with speed lam; a
// speed below 1e-10 of the system's fastest speed counts as zero and takes
// the mean (a rounding-level speed must not pick a side).
template <class R>
SHW_HD R upwind(R lam, R scale, R l, R r)
{
    const R z = 1e-10 * scale;
    return lam > z ? l : (lam < -z ? r : 0.5 * (l + r));
}

// The same choice as weights of the two sides, (1, 0), (0, 1) or (1/2, 1/2),
// for a speed shared by several problems (they sum to one, so a problem can
// be solved on the jump: x_r + w_l (x_l - x_r)).
template <class R>
SHW_HD void upwind_weights(R lam, R scale, R &wl, R &wr)
{
    const R z = 1e-10 * scale;
    wl = lam > z ? R(1.0) : (lam < -z ? R(0.0) : R(0.5));
    wr = lam > z ? R(0.0) : (lam < -z ? R(1.0) : R(0.5));
}

// Exact Godunov state of Burgers' equation at x/t = 0 (sec. 2.1.1, scalar case).
template <class R>
SHW_HD R burgers_state(R ul, R ur)
{
    if (ul > ur) {
        const R s = 0.5 * (ul + ur);
        return s > 0.0 ? ul : (s < 0.0 ? ur : s);
    }
    return ul >= 0.0 ? ul : (ur <= 0.0 ? ur : R(0.0));
}

} // namespace shw

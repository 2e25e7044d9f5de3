/*
 * recon.c -- SHWENO reconstruction of one scalar field on one cell.
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle; see shweno_oracle.h).
 *
 * The paper defers the reconstruction formulas to the simple-HWENO work it
 * cites (sec. 2.3) and fixes only the linear weights 0.994, 0.003, 0.003.
 * Reading used here (checked against the paper's error tables by the tests):
 *   - big stencil: the quartic p1 on the centre cell whose averages over cells
 *     -1, 0, +1 equal the given averages and whose integral of p1' over cells
 *     -1 and +1 equals the scaled derivative averages dx*V (sec. 2.4, eq. (vv));
 *   - two linear sub-stencils p2 (cells -1,0) and p3 (cells 0,+1);
 *   - smoothness indicators sum_{k>=1} int (d^k p/dxi^k)^2 over the cell;
 *   - simple-WENO ("Z"-type) weights with tau = ((|b1-b2|+|b1-b3|)/2)^2,
 *     w~_l = g_l (1 + tau/(beta_l + eps)), normalised;
 *   - final polynomial (w1/g1)(p1 - g2 p2 - g3 p3) + w2 p2 + w3 p3, used for
 *     the value and for every derivative (sec. 2.1.2: one set of weights and
 *     indicators for the function and all its derivatives).
 * Coordinates: xi = (x - x_j)/dx on [-1/2, 1/2].
 */
#include <math.h>
#include <string.h>
#include "shweno_oracle.h"

/* Gauss-Jordan inverse of an n x n row-major matrix (n <= 8) with partial
 * pivoting.  Returns 0 on success. */
int orc_invert(int n, const double *A, double *Ainv)
{
    double M[8][16];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            M[r][c] = (c < n) ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (M[piv][col] == 0.0) return 1;
        if (piv != col)
            for (int c = 0; c < 2 * n; ++c) {
                double t = M[col][c]; M[col][c] = M[piv][c]; M[piv][c] = t;
            }
        double d = M[col][col];
        for (int c = 0; c < 2 * n; ++c) M[col][c] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double f = M[r][col];
            if (f == 0.0) continue;
            for (int c = 0; c < 2 * n; ++c) M[r][c] -= f * M[col][c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Ainv[r * n + c] = M[r][n + c];
    return 0;
}

/* integral of xi^k over [lo, hi] */
static double mono_int(int k, double lo, double hi)
{
    return (pow(hi, k + 1) - pow(lo, k + 1)) / (k + 1);
}

/* The five conditions on the quartic, one row per condition, one column per
 * coefficient: average over cell l (l = -1, 0, +1) and jump p(l+1/2)-p(l-1/2)
 * over cells l = -1, +1.  Its inverse maps data to coefficients. */
static double big_inv[25];

/* built once when the library loads (so threads never race on it) */
__attribute__((constructor)) static void big_init(void)
{
    double A[25];
    const int lavg[3] = {-1, 0, 1};
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 5; ++k)
            A[r * 5 + k] = mono_int(k, lavg[r] - 0.5, lavg[r] + 0.5);
    const int lder[2] = {-1, 1};
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 5; ++k)
            A[(3 + r) * 5 + k] = pow(lder[r] + 0.5, k) - pow(lder[r] - 0.5, k);
    orc_invert(5, A, big_inv);
}

void orc_big_quartic(const double a[3], const double b[2], double c[5])
{
    const double d[5] = {a[0], a[1], a[2], b[0], b[1]};
    for (int k = 0; k < 5; ++k) {
        double s = 0.0;
        for (int r = 0; r < 5; ++r) s += big_inv[k * 5 + r] * d[r];
        c[k] = s;
    }
}

/* k-th derivative of sum c_i xi^i at xi */
double orc_poly_deriv(const double c[5], int k, double xi)
{
    double s = 0.0;
    for (int i = k; i < 5; ++i) {
        double f = 1.0;
        for (int t = 0; t < k; ++t) f *= (double)(i - t);
        s += c[i] * f * pow(xi, i - k);
    }
    return s;
}

double orc_smoothness(const double c[5])
{
    /* 4-point Gauss-Legendre on [-1/2,1/2] integrates (p')^2 (degree 6)
     * exactly. */
    const double s6 = sqrt(6.0 / 5.0);
    const double xn[2] = {sqrt(3.0 / 7.0 - 2.0 / 7.0 * s6), sqrt(3.0 / 7.0 + 2.0 / 7.0 * s6)};
    const double wn[2] = {(18.0 + sqrt(30.0)) / 36.0, (18.0 - sqrt(30.0)) / 36.0};
    double beta = 0.0;
    for (int k = 1; k <= 4; ++k)
        for (int q = 0; q < 2; ++q)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                double v = orc_poly_deriv(c, k, 0.5 * sgn * xn[q]);
                beta += 0.5 * wn[q] * v * v;
            }
    return beta;
}

static void linear_left(const double a[3], double c[5])
{
    memset(c, 0, 5 * sizeof(double));
    c[0] = a[1];
    c[1] = a[1] - a[0];
}

static void linear_right(const double a[3], double c[5])
{
    memset(c, 0, 5 * sizeof(double));
    c[0] = a[1];
    c[1] = a[2] - a[1];
}

void orc_weights(const orc_cfg *cfg, const double a[3], const double b[2], double w[3])
{
    double p[3][5];
    orc_big_quartic(a, b, p[0]);
    linear_left(a, p[1]);
    linear_right(a, p[2]);
    double beta[3];
    for (int l = 0; l < 3; ++l) beta[l] = orc_smoothness(p[l]);
    double tau = 0.5 * (fabs(beta[0] - beta[1]) + fabs(beta[0] - beta[2]));
    tau = tau * tau;
    double wt[3], sum = 0.0;
    for (int l = 0; l < 3; ++l) {
        wt[l] = cfg->lin_w[l] * (1.0 + tau / (beta[l] + cfg->eps));
        sum += wt[l];
    }
    for (int l = 0; l < 3; ++l) w[l] = wt[l] / sum;
}

void orc_combine(const orc_cfg *cfg, const double a[3], const double b[2],
                 const double w[3], double c[5])
{
    double p[3][5];
    orc_big_quartic(a, b, p[0]);
    linear_left(a, p[1]);
    linear_right(a, p[2]);
    const double *g = cfg->lin_w;
    for (int k = 0; k < 5; ++k)
        c[k] = w[0] / g[0] * (p[0][k] - g[1] * p[1][k] - g[2] * p[2][k])
             + w[1] * p[1][k] + w[2] * p[2][k];
}

void orc_recon_scalar(const orc_cfg *cfg, int mode, const double a[3],
                      const double b[2], double c[5])
{
    if (mode == ORC_W_LINEAR) {
        orc_big_quartic(a, b, c);
        return;
    }
    double w[3];
    orc_weights(cfg, a, b, w);
    orc_combine(cfg, a, b, w, c);
}

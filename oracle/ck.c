/*
 * ck.c -- the GRP at one interface point: leading term, linearised derivative
 * Riemann problems, and the Lax-Wendroff (Cauchy-Kovalevskaya) procedure.
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle; see shweno_oracle.h).
 *
 * The interface solution is carried as a truncated Taylor series in (x, y, t)
 * about the interface point, total degree <= 4: w[c][a][b][k] is the
 * coefficient of x^a y^b t^k of component c, so the time derivatives of
 * eq. (tay) are d^k W/dt^k = k! w[c][0][0][k].  The time layers follow from the
 * PDE W_t = -F(W)_x - G(W)_y, matched power by power (the componentwise
 * Lax-Wendroff procedure of sec. 2.1.2 and sec. 3.1, carried to fourth order):
 *   (k+1) w[a][b][k+1] = -((a+1) F[a+1][b][k] + (b+1) G[a][b+1][k]),
 * where F, G are the series of the fluxes of the current series of W.
 */
#include <math.h>
#include <string.h>
#include "shweno_oracle.h"

void orc_euler_eigen(double gamma, int dim, int dir, const double *W,
                     double *lam, double *R, double *L);
void orc_hllc_state(double gamma, int dim, const double *WL, const double *WR,
                    double *Wstar);

#define S(a, b, k) (((a) * 5 + (b)) * 5 + (k))
#define NS 125

/* h = f*g truncated at total degree 4 (and at y-degree bmax) */
static void ser_mul(int bmax, const double *f, const double *g, double *h)
{
    memset(h, 0, NS * sizeof(double));
    for (int a = 0; a <= 4; ++a)
        for (int b = 0; b <= bmax && a + b <= 4; ++b)
            for (int k = 0; a + b + k <= 4; ++k) {
                double s = 0.0;
                for (int a1 = 0; a1 <= a; ++a1)
                    for (int b1 = 0; b1 <= b; ++b1)
                        for (int k1 = 0; k1 <= k; ++k1)
                            s += f[S(a1, b1, k1)] * g[S(a - a1, b - b1, k - k1)];
                h[S(a, b, k)] = s;
            }
}

/* r = 1/f, truncated: r*f = 1 solved degree by degree */
static void ser_recip(int bmax, const double *f, double *r)
{
    memset(r, 0, NS * sizeof(double));
    r[0] = 1.0 / f[0];
    for (int d = 1; d <= 4; ++d)
        for (int a = 0; a <= d; ++a)
            for (int b = 0; b <= bmax && a + b <= d; ++b) {
                int k = d - a - b;
                double s = 0.0;
                for (int a1 = 0; a1 <= a; ++a1)
                    for (int b1 = 0; b1 <= b; ++b1)
                        for (int k1 = 0; k1 <= k; ++k1) {
                            if (a1 + b1 + k1 == 0) continue;
                            s += f[S(a1, b1, k1)] * r[S(a - a1, b - b1, k - k1)];
                        }
                r[S(a, b, k)] = -s * r[0];
            }
}

static void ser_axpy(double alpha, const double *x, double *y)
{
    for (int i = 0; i < NS; ++i) y[i] += alpha * x[i];
}

/* series of the fluxes F, G of the series W (m components) */
static void flux_series(const orc_cfg *cfg, int dim, const double *W,
                        double *F, double *G)
{
    int m = orc_ncomp(cfg->eq, dim);
    int bmax = dim == 2 ? 4 : 0;   /* a 1D series has no y terms */
    memset(F, 0, (size_t)m * NS * sizeof(double));
    memset(G, 0, (size_t)m * NS * sizeof(double));
    if (cfg->eq == ORC_ADVECTION) {
        ser_axpy(cfg->adv_a, W, F);
        if (dim == 2) ser_axpy(cfg->adv_b, W, G);
        return;
    }
    if (cfg->eq == ORC_BURGERS) {
        double sq[NS];
        ser_mul(bmax, W, W, sq);
        ser_axpy(0.5, sq, F);
        if (dim == 2) ser_axpy(0.5, sq, G);
        return;
    }
    const double gm1 = cfg->gamma - 1.0;
    double r[NS], u[NS], p[NS], Ep[NS], t[NS];
    ser_recip(bmax, W, r);
    if (dim == 1) {
        const double *mx = W + NS, *E = W + 2 * NS;
        ser_mul(bmax, mx, r, u);
        double mu[NS];
        ser_mul(bmax, mx, u, mu);
        for (int i = 0; i < NS; ++i) p[i] = gm1 * (E[i] - 0.5 * mu[i]);
        for (int i = 0; i < NS; ++i) Ep[i] = E[i] + p[i];
        memcpy(F, mx, NS * sizeof(double));
        for (int i = 0; i < NS; ++i) F[NS + i] = mu[i] + p[i];
        ser_mul(bmax, Ep, u, t);
        memcpy(F + 2 * NS, t, NS * sizeof(double));
        return;
    }
    const double *mx = W + NS, *my = W + 2 * NS, *E = W + 3 * NS;
    double v[NS], mu[NS], mv[NS], nv[NS];
    ser_mul(bmax, mx, r, u);
    ser_mul(bmax, my, r, v);
    ser_mul(bmax, mx, u, mu);   /* rho u^2 */
    ser_mul(bmax, my, v, nv);   /* rho v^2 */
    ser_mul(bmax, my, u, mv);   /* rho u v */
    for (int i = 0; i < NS; ++i) p[i] = gm1 * (E[i] - 0.5 * (mu[i] + nv[i]));
    for (int i = 0; i < NS; ++i) Ep[i] = E[i] + p[i];
    memcpy(F, mx, NS * sizeof(double));
    for (int i = 0; i < NS; ++i) F[NS + i] = mu[i] + p[i];
    memcpy(F + 2 * NS, mv, NS * sizeof(double));
    ser_mul(bmax, Ep, u, t);
    memcpy(F + 3 * NS, t, NS * sizeof(double));
    memcpy(G, my, NS * sizeof(double));
    memcpy(G + NS, mv, NS * sizeof(double));
    for (int i = 0; i < NS; ++i) G[2 * NS + i] = nv[i] + p[i];
    ser_mul(bmax, Ep, v, t);
    memcpy(G + 3 * NS, t, NS * sizeof(double));
}

void orc_ck_fill(const orc_cfg *cfg, int dim, double *w)
{
    int m = orc_ncomp(cfg->eq, dim);
    for (int c = 0; c < m; ++c)
        for (int a = 0; a <= 4; ++a)
            for (int b = 0; b <= 4; ++b)
                for (int k = 1; k <= 4; ++k) w[c * NS + S(a, b, k)] = 0.0;
    int bmax = dim == 2 ? 4 : 0;
    double F[4 * NS], G[4 * NS];
    for (int k = 0; k < 4; ++k) {
        flux_series(cfg, dim, w, F, G);
        for (int c = 0; c < m; ++c)
            for (int a = 0; a + k + 1 <= 4; ++a)
                for (int b = 0; b <= bmax && a + b + k + 1 <= 4; ++b)
                    w[c * NS + S(a, b, k + 1)] =
                        -((a + 1) * F[c * NS + S(a + 1, b, k)] +
                          (b + 1) * G[c * NS + S(a, b + 1, k)]) / (k + 1);
    }
}

/* Upwind solution at x/t = 0 of a linear Riemann problem with speed lam.
 * A speed smaller than ZERO_SPEED times the fastest speed of the system
 * (scale) counts as zero and takes the mean of both sides: a speed that is
 * zero in exact arithmetic (a wall, a symmetric collision) comes out of
 * rounding as +-1e-16 and must not pick a side. */
#define ZERO_SPEED 1e-10
static double upwind(double lam, double scale, double l, double r)
{
    if (lam > ZERO_SPEED * scale) return l;
    if (lam < -ZERO_SPEED * scale) return r;
    return 0.5 * (l + r);
}

static double fact(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* exact Godunov state of Burgers' equation at x/t = 0 */
static double burgers_state(double ul, double ur)
{
    if (ul > ur) {                       /* shock */
        double s = 0.5 * (ul + ur);
        if (s > 0.0) return ul;
        if (s < 0.0) return ur;
        return 0.5 * (ul + ur);
    }
    if (ul >= 0.0) return ul;            /* rarefaction */
    if (ur <= 0.0) return ur;
    return 0.0;
}

/*
 * GRP at one interface point with normal x.  JL, JR: spatial derivatives
 * d^{a+b}W/dx^a dy^b of the left and right reconstructions at the point,
 * index (a*5+b)*m + c for a+b<=4.  Output: series w (m*125).
 *   leading term: exact (scalar) or HLLC (Euler) Riemann state (sec. 2.1.1);
 *   each derivative: linear Riemann problem with the Jacobian at the leading
 *     term, solved by upwinding every characteristic field (eq. (lineq) /
 *     (lineq2d); a zero speed takes the mean of both sides, a reading);
 *   time layers: orc_ck_fill.
 */
void orc_grp_face(const orc_cfg *cfg, int dim, const double *JL,
                  const double *JR, double *w)
{
    int m = orc_ncomp(cfg->eq, dim);
    memset(w, 0, (size_t)m * NS * sizeof(double));
    double Ws[4], lam[4], R[16], L[16];
    if (cfg->eq == ORC_EULER) {
        orc_hllc_state(cfg->gamma, dim, JL, JR, Ws);
        orc_euler_eigen(cfg->gamma, dim, 0, Ws, lam, R, L);
    } else if (cfg->eq == ORC_BURGERS) {
        Ws[0] = burgers_state(JL[0], JR[0]);
        lam[0] = Ws[0]; R[0] = 1.0; L[0] = 1.0;
    } else {
        Ws[0] = upwind(cfg->adv_a, fabs(cfg->adv_a), JL[0], JR[0]);
        lam[0] = cfg->adv_a; R[0] = 1.0; L[0] = 1.0;
    }
    for (int c = 0; c < m; ++c) w[c * NS + S(0, 0, 0)] = Ws[c];
    double scale = 0.0;
    for (int s = 0; s < m; ++s) scale = fmax(scale, fabs(lam[s]));
    int bmax = dim == 2 ? 4 : 0;
    for (int a = 0; a <= 4; ++a)
        for (int b = 0; b <= bmax && a + b <= 4; ++b) {
            if (a + b == 0) continue;
            const double *DL = JL + (a * 5 + b) * m, *DR = JR + (a * 5 + b) * m;
            double ch[4];
            for (int s = 0; s < m; ++s) {
                double l = 0.0, r = 0.0;
                for (int c = 0; c < m; ++c) {
                    l += L[s * m + c] * DL[c];
                    r += L[s * m + c] * DR[c];
                }
                ch[s] = upwind(lam[s], scale, l, r);
            }
            for (int c = 0; c < m; ++c) {
                double d = 0.0;
                for (int s = 0; s < m; ++s) d += R[c * m + s] * ch[s];
                w[c * NS + S(a, b, 0)] = d / (fact(a) * fact(b));
            }
        }
    orc_ck_fill(cfg, dim, w);
}

/*
 * step.c -- one ADER-SHWENO time step in 1D and 2D, the CFL step size, and
 * the time loop.
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle; see shweno_oracle.h).
 *
 * Order of work follows the algorithm of sec. 4 (Steps 1-5): reconstruct
 * every cell, solve the GRP at every interface point (leading term, derivative
 * Riemann problems, Lax-Wendroff), integrate the flux in time (and along the
 * edge in 2D), update the averages (eq. (cons) / the 2D form in sec. 3) and the
 * derivative averages from the interface values at t_{n+1} (eqs. (derave),
 * (tay1d), (derave2d), (taylor2dtime)).
 *
 * Readings (the paper leaves these open):
 *   - time rule and edge rule: 4-point Gauss-Lobatto (Remark 2 and sec. 3.3
 *     name Gauss-Lobatto; four points integrate the degree-4 Taylor state's
 *     flux to the scheme's order), nodes {0, (1-1/sqrt5)/2, (1+1/sqrt5)/2, 1},
 *     weights {1,5,5,1}/12;
 *   - Euler: reconstruction of characteristic fields, eigenvectors of the
 *     Jacobian in the sweep direction at the cell's own average;
 *   - 2D: stage 1 (transverse) reconstructs {W,Y} and {V,Z} with one weight
 *     set computed from the {W,Y} data; stage 2 computes its weights from the
 *     order-0 data and reuses them for the transverse derivatives;
 *   - the mixed average Z is the mean of the corner formula of eq. (derave2d)
 *     evaluated with x-interface values and with y-interface values;
 *   - CFL: 1D dt = cfl dx / max(|u|+c), 2D dt = cfl / max((|u|+c)/dx +
 *     (|v|+c)/dy), both over the cell averages at t_n;
 *   - boundary ghost cells: periodic wrap; transmissive copies the nearest
 *     average and sets every average containing a normal derivative to zero;
 *     reflective mirrors, with the sign of odd quantities flipped.
 * The y-direction half of the 2D step runs the x-direction procedure on the
 * transposed state (x<->y, V<->Y, momentum components swapped): the Euler
 * equations are invariant under that map.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "shweno_oracle.h"

void orc_euler_flux_x(double gamma, int dim, const double *W, double *F);
void orc_grp_face(const orc_cfg *cfg, int dim, const double *JL,
                  const double *JR, double *w);
double orc_poly_deriv(const double c[5], int k, double xi);

#define NS 125
#define SI(a, b, k) (((a) * 5 + (b)) * 5 + (k))

static void lobatto(double node[4], double wt[4])
{
    double h = 0.5 / sqrt(5.0);
    node[0] = -0.5; node[1] = -h; node[2] = h; node[3] = 0.5;
    wt[0] = 1.0 / 12.0; wt[1] = 5.0 / 12.0; wt[2] = 5.0 / 12.0; wt[3] = 1.0 / 12.0;
}

static double ipow(double x, int k)
{
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

/* physical flux in the x direction of a point state */
static void point_flux(const orc_cfg *cfg, int dim, const double *W, double *F)
{
    if (cfg->eq == ORC_EULER) orc_euler_flux_x(cfg->gamma, dim, W, F);
    else if (cfg->eq == ORC_BURGERS) F[0] = 0.5 * W[0] * W[0];
    else F[0] = cfg->adv_a * W[0];
}

static int nonphysical(const orc_cfg *cfg, int dim, const double *W)
{
    int m = orc_ncomp(cfg->eq, dim);
    for (int c = 0; c < m; ++c)
        if (!isfinite(W[c])) return 1;
    if (cfg->eq != ORC_EULER) return 0;
    double rho = W[0];
    if (!(rho > 0.0)) return 1;
    double ke = 0.5 * W[1] * W[1] / rho;
    if (dim == 2) ke += 0.5 * W[2] * W[2] / rho;
    double p = (cfg->gamma - 1.0) * (W[m - 1] - ke);
    return !(p > 0.0);
}

/* sound speed plus |normal velocity| (Euler), or the scalar wave speed */
static double wave_speed(const orc_cfg *cfg, int dim, int dir, const double *W)
{
    if (cfg->eq == ORC_ADVECTION) return fabs(dir == 0 ? cfg->adv_a : cfg->adv_b);
    if (cfg->eq == ORC_BURGERS) return fabs(W[0]);
    int m = orc_ncomp(cfg->eq, dim);
    double rho = W[0], u = W[1] / rho, v = dim == 2 ? W[2] / rho : 0.0;
    double p = (cfg->gamma - 1.0) * (W[m - 1] - 0.5 * rho * (u * u + v * v));
    double c = sqrt(cfg->gamma * p / rho);
    return fabs(dir == 0 ? u : v) + c;
}

/* ------------------------------------------------------------------------- */
/* 1D                                                                        */
/* ------------------------------------------------------------------------- */

/* index of the interior cell a ghost cell takes its data from */
static int source_index(int bc, int n, int j)
{
    if (j >= 0 && j < n) return j;
    if (bc == ORC_BC_PERIODIC) return ((j % n) + n) % n;
    if (bc == ORC_BC_TRANSMISSIVE) return j < 0 ? 0 : n - 1;
    return j < 0 ? -1 - j : 2 * n - 1 - j;   /* reflective: mirror */
}

/* averages of cell j (W: value, V: x-derivative), ghosts by the BCs
 * (also used by the gate's features and labels) */
void orc_cell1d(const orc_cfg *cfg, int n, const double *st, int j, double *W, double *V)
{
    int m = orc_ncomp(cfg->eq, 1);
    int bc = j < 0 ? cfg->bc[0] : cfg->bc[1];
    int s = source_index(bc, n, j);
    for (int c = 0; c < m; ++c) {
        W[c] = st[c * n + s];
        V[c] = st[(m + c) * n + s];
    }
    if (j >= 0 && j < n) return;
    if (bc == ORC_BC_TRANSMISSIVE) {
        for (int c = 0; c < m; ++c) V[c] = 0.0;
    } else if (bc == ORC_BC_REFLECTIVE) {
        for (int c = 0; c < m; ++c) {
            double par = (cfg->eq == ORC_EULER && c == 1) ? -1.0 : 1.0;
            W[c] *= par;
            V[c] *= -par;
        }
    }
}

static int full_recon(const orc_cfg *cfg, const unsigned char *flags, int src)
{
    if (cfg->weights == ORC_W_NONLINEAR) return 1;
    if (cfg->weights == ORC_W_LINEAR) return 0;
    return flags[src] != 0;
}

/* Reconstruction polynomials (per component, in xi) of cell j. */
static void recon_cell1d(const orc_cfg *cfg, int n, double dx, const double *st,
                         const unsigned char *flags, int j, double P[4][5])
{
    int m = orc_ncomp(cfg->eq, 1);
    double W[3][4], V[3][4];
    for (int l = 0; l < 3; ++l) orc_cell1d(cfg, n, st, j - 1 + l, W[l], V[l]);
    int bc = j < 0 ? cfg->bc[0] : cfg->bc[1];
    int full = full_recon(cfg, flags, source_index(bc, n, j));
    if (cfg->eq == ORC_EULER && cfg->charwise && full) {
        double lam[3], R[9], L[9], ch[3][5];
        orc_euler_eigen(cfg->gamma, 1, 0, W[1], lam, R, L);
        for (int s = 0; s < m; ++s) {
            double a[3], b[2];
            for (int l = 0; l < 3; ++l) {
                a[l] = 0.0;
                for (int c = 0; c < m; ++c) a[l] += L[s * m + c] * W[l][c];
            }
            for (int l = 0; l < 2; ++l) {
                b[l] = 0.0;
                for (int c = 0; c < m; ++c) b[l] += L[s * m + c] * V[2 * l][c];
                b[l] *= dx;
            }
            orc_recon_scalar(cfg, ORC_W_NONLINEAR, a, b, ch[s]);
        }
        for (int c = 0; c < m; ++c)
            for (int k = 0; k < 5; ++k) {
                P[c][k] = 0.0;
                for (int s = 0; s < m; ++s) P[c][k] += R[c * m + s] * ch[s][k];
            }
        return;
    }
    for (int c = 0; c < m; ++c) {
        double a[3] = {W[0][c], W[1][c], W[2][c]};
        double b[2] = {dx * V[0][c], dx * V[2][c]};
        orc_recon_scalar(cfg, full ? ORC_W_NONLINEAR : ORC_W_LINEAR, a, b, P[c]);
    }
}

/* Positivity safeguard (an addition to the paper's scheme, which has no
 * limiter; used only when cfg->positivity is set).  A cell is troubled when
 * its update from the face fluxes Fh (Step 5) would be non-physical.  Every
 * face next to a troubled cell takes the first-order HLLE flux of the two
 * cell averages at t_n instead (ghost cells by the boundary conditions;
 * Einfeldt's wave-speed bounds, with which the first-order scheme keeps
 * density and pressure positive), its state at x/t = 0 standing for the face
 * value at t_{n+1} in the derivative averages.  Both cells of a face see the
 * same flux, so the update stays conservative.  One round: a cell that is
 * still non-physical fails the step. */
static void first_order_faces(const orc_cfg *cfg, int n, double dx, double dt,
                              const double *in, double *Fh, double *We)
{
    int m = orc_ncomp(cfg->eq, 1);
    unsigned char *trouble = malloc((size_t)n);
    for (int j = 0; j < n; ++j) {
        double Wn[4];
        for (int c = 0; c < m; ++c)
            Wn[c] = in[c * n + j] - dt / dx * (Fh[(j + 1) * m + c] - Fh[j * m + c]);
        trouble[j] = (unsigned char)nonphysical(cfg, 1, Wn);
    }
    for (int f = 0; f <= n; ++f) {
        /* the cells on both sides; a ghost stands for the cell it copies */
        int l = source_index(cfg->bc[0], n, f - 1);
        int r = source_index(cfg->bc[1], n, f);
        if (!trouble[l] && !trouble[r]) continue;
        double WL[4], VL[4], WR[4], VR[4], Ws[4], F[4];
        orc_cell1d(cfg, n, in, f - 1, WL, VL);
        orc_cell1d(cfg, n, in, f, WR, VR);
        orc_hlle(cfg->gamma, 1, WL, WR, F, Ws);
        for (int c = 0; c < m; ++c) {
            Fh[f * m + c] = F[c];
            We[f * m + c] = Ws[c];
        }
    }
    free(trouble);
}

int orc_step1d(const orc_cfg *cfg, int n, double dx, double dt,
               const double *in, double *out, const unsigned char *flags)
{
    int m = orc_ncomp(cfg->eq, 1);
    double tn[4], tw[4];
    lobatto(tn, tw);
    /* Step 1: reconstruction of cells -1..n (each face needs both sides) */
    double (*P)[4][5] = malloc(sizeof(double[4][5]) * (size_t)(n + 2));
    for (int j = -1; j <= n; ++j) recon_cell1d(cfg, n, dx, in, flags, j, P[j + 1]);
    /* Steps 2-4: GRP and time-integrated flux at faces f = j+1/2, j=-1..n-1 */
    double *Fh = malloc(sizeof(double) * (size_t)(n + 1) * m);
    double *We = malloc(sizeof(double) * (size_t)(n + 1) * m);
    for (int f = 0; f <= n; ++f) {
        const double (*PL)[5] = P[f];       /* cell f-1, right edge */
        const double (*PR)[5] = P[f + 1];   /* cell f, left edge */
        double JL[25 * 4], JR[25 * 4], w[4 * NS];
        memset(JL, 0, sizeof JL);
        memset(JR, 0, sizeof JR);
        for (int a = 0; a <= 4; ++a)
            for (int c = 0; c < m; ++c) {
                JL[(a * 5) * m + c] = orc_poly_deriv(PL[c], a, 0.5) / ipow(dx, a);
                JR[(a * 5) * m + c] = orc_poly_deriv(PR[c], a, -0.5) / ipow(dx, a);
            }
        orc_grp_face(cfg, 1, JL, JR, w);
        double acc[4] = {0, 0, 0, 0};
        for (int al = 0; al < 4; ++al) {
            double tau = (tn[al] + 0.5) * dt, Wt[4], F[4];
            for (int c = 0; c < m; ++c) {
                Wt[c] = 0.0;
                for (int k = 0; k <= 4; ++k) Wt[c] += w[c * NS + SI(0, 0, k)] * ipow(tau, k);
            }
            point_flux(cfg, 1, Wt, F);
            for (int c = 0; c < m; ++c) acc[c] += tw[al] * F[c];
            if (al == 3)
                for (int c = 0; c < m; ++c) We[f * m + c] = Wt[c];
        }
        for (int c = 0; c < m; ++c) Fh[f * m + c] = acc[c];
    }
    if (cfg->positivity && cfg->eq == ORC_EULER) first_order_faces(cfg, n, dx, dt, in, Fh, We);
    /* Step 5: update of averages and derivative averages */
    int bad = 0;
    for (int j = 0; j < n; ++j) {
        double Wn[4];
        for (int c = 0; c < m; ++c) {
            Wn[c] = in[c * n + j] - dt / dx * (Fh[(j + 1) * m + c] - Fh[j * m + c]);
            out[c * n + j] = Wn[c];
            out[(m + c) * n + j] = (We[(j + 1) * m + c] - We[j * m + c]) / dx;
        }
        bad |= nonphysical(cfg, 1, Wn);
    }
    free(P); free(Fh); free(We);
    return bad;
}

double orc_dt1d(const orc_cfg *cfg, int n, double dx, double cfl, const double *st)
{
    int m = orc_ncomp(cfg->eq, 1);
    double smax = 0.0;
    for (int j = 0; j < n; ++j) {
        double W[4];
        for (int c = 0; c < m; ++c) W[c] = st[c * n + j];
        if (nonphysical(cfg, 1, W)) return -1.0;
        double s = wave_speed(cfg, 1, 0, W);
        if (s > smax) smax = s;
    }
    return cfl * dx / smax;
}

int orc_advance1d(const orc_cfg *cfg, int n, double dx, double cfl, double T,
                  long max_steps, double *st, double *t, long *steps)
{
    int m = orc_ncomp(cfg->eq, 1);
    double *tmp = malloc(sizeof(double) * 2 * m * (size_t)n);
    int bad = 0;
    while (*t < T && *steps < max_steps) {
        double dt = orc_dt1d(cfg, n, dx, cfl, st);
        if (dt < 0) { bad = 1; break; }
        int last = 0;
        if (dt >= T - *t) { dt = T - *t; last = 1; }
        bad = orc_step1d(cfg, n, dx, dt, st, tmp, NULL);
        memcpy(st, tmp, sizeof(double) * 2 * m * (size_t)n);
        *t = last ? T : *t + dt;
        ++*steps;
        if (bad) break;
    }
    free(tmp);
    return bad;
}

/* ------------------------------------------------------------------------- */
/* 2D                                                                        */
/* ------------------------------------------------------------------------- */

/* the four averages (W, V, Y, Z; m components each) of cell (i, j), ghosts by
 * the boundary conditions (also used by the gate's features) */
void orc_cell2d(const orc_cfg *cfg, int nx, int ny, const double *st, int i, int j,
                double Q[4][4])
{
    int m = orc_ncomp(cfg->eq, 2);
    int bx = i < 0 ? cfg->bc[0] : cfg->bc[1];
    int by = j < 0 ? cfg->bc[2] : cfg->bc[3];
    int si = source_index(bx, nx, i), sj = source_index(by, ny, j);
    size_t plane = (size_t)nx * ny;
    for (int q = 0; q < 4; ++q)
        for (int c = 0; c < m; ++c)
            Q[q][c] = st[(q * m + c) * plane + (size_t)sj * nx + si];
    int ghost_x = !(i >= 0 && i < nx), ghost_y = !(j >= 0 && j < ny);
    if (ghost_x) {
        if (bx == ORC_BC_TRANSMISSIVE) {
            for (int c = 0; c < m; ++c) { Q[1][c] = 0.0; Q[3][c] = 0.0; }
        } else if (bx == ORC_BC_REFLECTIVE) {
            for (int c = 0; c < m; ++c) {
                double par = (cfg->eq == ORC_EULER && c == 1) ? -1.0 : 1.0;
                Q[0][c] *= par; Q[1][c] *= -par; Q[2][c] *= par; Q[3][c] *= -par;
            }
        }
    }
    if (ghost_y) {
        if (by == ORC_BC_TRANSMISSIVE) {
            for (int c = 0; c < m; ++c) { Q[2][c] = 0.0; Q[3][c] = 0.0; }
        } else if (by == ORC_BC_REFLECTIVE) {
            for (int c = 0; c < m; ++c) {
                double par = (cfg->eq == ORC_EULER && c == 2) ? -1.0 : 1.0;
                Q[0][c] *= par; Q[1][c] *= par; Q[2][c] *= -par; Q[3][c] *= -par;
            }
        }
    }
}

static int flag2d(const orc_cfg *cfg, int nx, int ny, const unsigned char *flags,
                  int i, int j)
{
    int si = source_index(i < 0 ? cfg->bc[0] : cfg->bc[1], nx, i);
    int sj = source_index(j < 0 ? cfg->bc[2] : cfg->bc[3], ny, j);
    return full_recon(cfg, flags, sj * nx + si);
}

/*
 * Reconstruct data sets that share one weight set: nset scalar data sets
 * (a[set][3], b[set][2]) per component; weights from set 0.  Characteristic
 * fields of the Jacobian in direction dir at Wc when requested.  Output:
 * polynomials P[set][c][5] in conservative components.
 */
static void recon_shared(const orc_cfg *cfg, int full, int dir, const double *Wc,
                         int nset, double a[][3][4], double b[][2][4],
                         double P[][4][5])
{
    int m = orc_ncomp(cfg->eq, 2);
    if (!full) {
        for (int s = 0; s < nset; ++s)
            for (int c = 0; c < m; ++c) {
                double aa[3] = {a[s][0][c], a[s][1][c], a[s][2][c]};
                double bb[2] = {b[s][0][c], b[s][1][c]};
                orc_big_quartic(aa, bb, P[s][c]);
            }
        return;
    }
    double lam[4], R[16], L[16];
    int proj = cfg->eq == ORC_EULER && cfg->charwise;
    if (proj) orc_euler_eigen(cfg->gamma, 2, dir, Wc, lam, R, L);
    double ch[8][4][5];
    for (int f = 0; f < m; ++f) {
        double aa[8][3], bb[8][2];
        for (int s = 0; s < nset; ++s) {
            for (int l = 0; l < 3; ++l) {
                if (!proj) { aa[s][l] = a[s][l][f]; continue; }
                aa[s][l] = 0.0;
                for (int c = 0; c < m; ++c) aa[s][l] += L[f * m + c] * a[s][l][c];
            }
            for (int l = 0; l < 2; ++l) {
                if (!proj) { bb[s][l] = b[s][l][f]; continue; }
                bb[s][l] = 0.0;
                for (int c = 0; c < m; ++c) bb[s][l] += L[f * m + c] * b[s][l][c];
            }
        }
        double w[3];
        orc_weights(cfg, aa[0], bb[0], w);
        for (int s = 0; s < nset; ++s) orc_combine(cfg, aa[s], bb[s], w, ch[s][f]);
    }
    for (int s = 0; s < nset; ++s)
        for (int c = 0; c < m; ++c)
            for (int k = 0; k < 5; ++k) {
                if (!proj) { P[s][c][k] = ch[s][c][k]; continue; }
                P[s][c][k] = 0.0;
                for (int f = 0; f < m; ++f) P[s][c][k] += R[c * m + f] * ch[s][f][k];
            }
}

/* stage 1 result of one cell: A[g][n][c] = d^n/dy^n of the x-average of W at
 * the edge node g, B[g][n][c] the same for W_x */
typedef struct { double A[4][5][4], B[4][5][4]; } stage1_t;
/* stage 2 result of one cell: J[side][g][(a*5+n)*m + c], side 0: xi=-1/2,
 * side 1: xi=+1/2; d^{a+n}W/dx^a dy^n at edge node g */
typedef struct { double J[2][4][25 * 4]; } stage2_t;

static void stage1(const orc_cfg *cfg, int nx, int ny, double dy,
                   const double *st, const unsigned char *flags, int i, int j,
                   stage1_t *out)
{
    int m = orc_ncomp(cfg->eq, 2);
    double Q[3][4][4];
    for (int l = 0; l < 3; ++l) orc_cell2d(cfg, nx, ny, st, i, j - 1 + l, Q[l]);
    double a[2][3][4], b[2][2][4], P[2][4][5];
    for (int c = 0; c < m; ++c) {
        for (int l = 0; l < 3; ++l) {
            a[0][l][c] = Q[l][0][c];      /* W averages */
            a[1][l][c] = Q[l][1][c];      /* V averages */
        }
        b[0][0][c] = dy * Q[0][2][c]; b[0][1][c] = dy * Q[2][2][c];   /* Y */
        b[1][0][c] = dy * Q[0][3][c]; b[1][1][c] = dy * Q[2][3][c];   /* Z */
    }
    int full = flag2d(cfg, nx, ny, flags, i, j);
    recon_shared(cfg, full, 1, Q[1][0], 2, a, b, P);
    double node[4], wt[4];
    lobatto(node, wt);
    for (int g = 0; g < 4; ++g)
        for (int n = 0; n <= 4; ++n)
            for (int c = 0; c < m; ++c) {
                out->A[g][n][c] = orc_poly_deriv(P[0][c], n, node[g]) / ipow(dy, n);
                out->B[g][n][c] = orc_poly_deriv(P[1][c], n, node[g]) / ipow(dy, n);
            }
}

static void stage2(const orc_cfg *cfg, int nx, int ny, double dx,
                   const double *st, const unsigned char *flags, int i, int j,
                   const stage1_t *s1m, const stage1_t *s10, const stage1_t *s1p,
                   stage2_t *out)
{
    int m = orc_ncomp(cfg->eq, 2);
    double Q[4][4];
    orc_cell2d(cfg, nx, ny, st, i, j, Q);
    int full = flag2d(cfg, nx, ny, flags, i, j);
    memset(out, 0, sizeof *out);
    for (int g = 0; g < 4; ++g) {
        double a[5][3][4], b[5][2][4], P[5][4][5];
        for (int n = 0; n <= 4; ++n)
            for (int c = 0; c < m; ++c) {
                a[n][0][c] = s1m->A[g][n][c];
                a[n][1][c] = s10->A[g][n][c];
                a[n][2][c] = s1p->A[g][n][c];
                b[n][0][c] = dx * s1m->B[g][n][c];
                b[n][1][c] = dx * s1p->B[g][n][c];
            }
        recon_shared(cfg, full, 0, Q[0], 5, a, b, P);
        for (int n = 0; n <= 4; ++n)
            for (int aa = 0; aa + n <= 4; ++aa)
                for (int c = 0; c < m; ++c) {
                    out->J[0][g][(aa * 5 + n) * m + c] =
                        orc_poly_deriv(P[n][c], aa, -0.5) / ipow(dx, aa);
                    out->J[1][g][(aa * 5 + n) * m + c] =
                        orc_poly_deriv(P[n][c], aa, 0.5) / ipow(dx, aa);
                }
    }
}

/*
 * x-direction interfaces of the whole grid.  Face f (f = 0..nx) of row j lies
 * between cells f-1 and f.  Fh[(j*(nx+1)+f)*m + c]: flux averaged over the
 * time step and the edge (eq. (fx2d) divided by dy); We[((j*(nx+1)+f)*4+g)*m
 * + c]: the interface state at t_{n+1} at edge node g.
 */
static void xsweep(const orc_cfg *cfg, int nx, int ny, double dx, double dy,
                   double dt, const double *st, const unsigned char *flags,
                   double *Fh, double *We)
{
    int m = orc_ncomp(cfg->eq, 2);
    double tn[4], tw[4];
    lobatto(tn, tw);
    /* rows are independent: one row per thread */
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < ny; ++j) {
        stage1_t *s1 = malloc(sizeof(stage1_t) * (size_t)(nx + 4));
        stage2_t *s2 = malloc(sizeof(stage2_t) * (size_t)(nx + 2));
        for (int i = -2; i <= nx + 1; ++i)
            stage1(cfg, nx, ny, dy, st, flags, i, j, &s1[i + 2]);
        for (int i = -1; i <= nx; ++i)
            stage2(cfg, nx, ny, dx, st, flags, i, j, &s1[i + 1], &s1[i + 2],
                   &s1[i + 3], &s2[i + 1]);
        for (int f = 0; f <= nx; ++f) {
            double acc[4] = {0, 0, 0, 0};
            for (int g = 0; g < 4; ++g) {
                double w[4 * NS];
                orc_grp_face(cfg, 2, s2[f].J[1][g], s2[f + 1].J[0][g], w);
                for (int al = 0; al < 4; ++al) {
                    double tau = (tn[al] + 0.5) * dt, Wt[4], F[4];
                    for (int c = 0; c < m; ++c) {
                        Wt[c] = 0.0;
                        for (int k = 0; k <= 4; ++k)
                            Wt[c] += w[c * NS + SI(0, 0, k)] * ipow(tau, k);
                    }
                    if (cfg->eq == ORC_EULER) orc_euler_flux_x(cfg->gamma, 2, Wt, F);
                    else if (cfg->eq == ORC_BURGERS) F[0] = 0.5 * Wt[0] * Wt[0];
                    else F[0] = cfg->adv_a * Wt[0];
                    for (int c = 0; c < m; ++c) acc[c] += tw[g] * tw[al] * F[c];
                    if (al == 3)
                        for (int c = 0; c < m; ++c)
                            We[(((size_t)j * (nx + 1) + f) * 4 + g) * m + c] = Wt[c];
                }
            }
            for (int c = 0; c < m; ++c) Fh[((size_t)j * (nx + 1) + f) * m + c] = acc[c];
        }
        free(s1); free(s2);
    }
}

static int comp_swap(const orc_cfg *cfg, int c)
{
    if (cfg->eq != ORC_EULER) return c;
    return c == 1 ? 2 : (c == 2 ? 1 : c);
}

/* The 2D positivity safeguard (cfg->positivity; an addition, as in 1D): a
 * cell is troubled when its update from the face data would be non-physical;
 * every x- and y-face next to a troubled cell takes the first-order HLLE flux
 * of the two cell averages at t_n (ghosts by the boundary conditions; a
 * y-face in the frame with x and y exchanged, in which its arrays are kept),
 * and the HLLE state at x/t = 0 stands for the face value at t_{n+1} at all
 * four edge nodes.  Fh/Wx: x-faces; Gt/Wyt: y-faces, transposed frame. */
static void first_order_faces2d(const orc_cfg *cfg, int nx, int ny, double dx, double dy,
                                double dt, const double *in, double *Fh, double *Wx,
                                double *Gt, double *Wyt)
{
    const int m = 4;
    size_t plane = (size_t)nx * ny;
    unsigned char *trouble = malloc(plane);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double Wn[4];
            size_t o = (size_t)j * nx + i;
            for (int c = 0; c < m; ++c) {
                int cs = comp_swap(cfg, c);
                Wn[c] = in[c * plane + o]
                      - dt / dx * (Fh[((size_t)j * (nx + 1) + i + 1) * m + c]
                                   - Fh[((size_t)j * (nx + 1) + i) * m + c])
                      - dt / dy * (Gt[((size_t)i * (ny + 1) + j + 1) * m + cs]
                                   - Gt[((size_t)i * (ny + 1) + j) * m + cs]);
            }
            trouble[o] = (unsigned char)nonphysical(cfg, 2, Wn);
        }
    /* x-faces: face f of row j between cells f-1 and f */
    for (int j = 0; j < ny; ++j)
        for (int f = 0; f <= nx; ++f) {
            int l = source_index(cfg->bc[0], nx, f - 1), r = source_index(cfg->bc[1], nx, f);
            if (!trouble[(size_t)j * nx + l] && !trouble[(size_t)j * nx + r]) continue;
            double QL[4][4], QR[4][4], F[4], Ws[4];
            orc_cell2d(cfg, nx, ny, in, f - 1, j, QL);
            orc_cell2d(cfg, nx, ny, in, f, j, QR);
            orc_hlle(cfg->gamma, 2, QL[0], QR[0], F, Ws);
            for (int c = 0; c < m; ++c) {
                Fh[((size_t)j * (nx + 1) + f) * m + c] = F[c];
                for (int g = 0; g < 4; ++g)
                    Wx[(((size_t)j * (nx + 1) + f) * 4 + g) * m + c] = Ws[c];
            }
        }
    /* y-faces: face f of column i between cells f-1 and f, in the frame with
     * x and y exchanged (momenta swapped) */
    for (int i = 0; i < nx; ++i)
        for (int f = 0; f <= ny; ++f) {
            int l = source_index(cfg->bc[2], ny, f - 1), r = source_index(cfg->bc[3], ny, f);
            if (!trouble[(size_t)l * nx + i] && !trouble[(size_t)r * nx + i]) continue;
            double QL[4][4], QR[4][4], WL[4], WR[4], F[4], Ws[4];
            orc_cell2d(cfg, nx, ny, in, i, f - 1, QL);
            orc_cell2d(cfg, nx, ny, in, i, f, QR);
            for (int c = 0; c < m; ++c) {
                WL[comp_swap(cfg, c)] = QL[0][c];
                WR[comp_swap(cfg, c)] = QR[0][c];
            }
            orc_hlle(cfg->gamma, 2, WL, WR, F, Ws);
            for (int c = 0; c < m; ++c) {
                Gt[((size_t)i * (ny + 1) + f) * m + c] = F[c];
                for (int g = 0; g < 4; ++g)
                    Wyt[(((size_t)i * (ny + 1) + f) * 4 + g) * m + c] = Ws[c];
            }
        }
    free(trouble);
}

int orc_step2d(const orc_cfg *cfg, int nx, int ny, double dx, double dy,
               double dt, const double *in, double *out,
               const unsigned char *flags)
{
    int m = orc_ncomp(cfg->eq, 2);
    size_t plane = (size_t)nx * ny;
    double tn[4], tw[4];
    lobatto(tn, tw);
    /* x interfaces */
    double *Fh = malloc(sizeof(double) * (size_t)ny * (nx + 1) * m);
    double *Wx = malloc(sizeof(double) * (size_t)ny * (nx + 1) * 4 * m);
    xsweep(cfg, nx, ny, dx, dy, dt, in, flags, Fh, Wx);
    /* y interfaces: the x procedure on the transposed problem */
    orc_cfg ct = *cfg;
    ct.bc[0] = cfg->bc[2]; ct.bc[1] = cfg->bc[3];
    ct.bc[2] = cfg->bc[0]; ct.bc[3] = cfg->bc[1];
    ct.adv_a = cfg->adv_b; ct.adv_b = cfg->adv_a;
    double *tst = malloc(sizeof(double) * 4 * m * plane);
    unsigned char *tfl = flags ? malloc(plane) : NULL;
    const int qmap[4] = {0, 2, 1, 3};
    for (int q = 0; q < 4; ++q)
        for (int c = 0; c < m; ++c)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i)
                    tst[(qmap[q] * m + comp_swap(cfg, c)) * plane + (size_t)i * ny + j] =
                        in[(q * m + c) * plane + (size_t)j * nx + i];
    if (tfl)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) tfl[(size_t)i * ny + j] = flags[(size_t)j * nx + i];
    double *Gt = malloc(sizeof(double) * (size_t)nx * (ny + 1) * m);
    double *Wyt = malloc(sizeof(double) * (size_t)nx * (ny + 1) * 4 * m);
    xsweep(&ct, ny, nx, dy, dx, dt, tst, tfl, Gt, Wyt);
    if (cfg->positivity && cfg->eq == ORC_EULER)
        first_order_faces2d(cfg, nx, ny, dx, dy, dt, in, Fh, Wx, Gt, Wyt);
    /* update (Step 5) */
    int bad = 0;
#define FH(j, f, c) Fh[((size_t)(j) * (nx + 1) + (f)) * m + (c)]
#define WX(j, f, g, c) Wx[(((size_t)(j) * (nx + 1) + (f)) * 4 + (g)) * m + (c)]
#define GH(i, f, c) Gt[((size_t)(i) * (ny + 1) + (f)) * m + comp_swap(cfg, c)]
#define WY(i, f, g, c) Wyt[(((size_t)(i) * (ny + 1) + (f)) * 4 + (g)) * m + comp_swap(cfg, c)]
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double Wn[4];
            size_t o = (size_t)j * nx + i;
            for (int c = 0; c < m; ++c) {
                double Wb = in[c * plane + o];
                Wn[c] = Wb - dt / dx * (FH(j, i + 1, c) - FH(j, i, c))
                           - dt / dy * (GH(i, j + 1, c) - GH(i, j, c));
                double V = 0.0, Y = 0.0;
                for (int g = 0; g < 4; ++g) {
                    V += tw[g] * (WX(j, i + 1, g, c) - WX(j, i, g, c));
                    Y += tw[g] * (WY(i, j + 1, g, c) - WY(i, j, g, c));
                }
                double Zx = WX(j, i + 1, 3, c) - WX(j, i, 3, c)
                          - WX(j, i + 1, 0, c) + WX(j, i, 0, c);
                double Zy = WY(i, j + 1, 3, c) - WY(i, j + 1, 0, c)
                          - WY(i, j, 3, c) + WY(i, j, 0, c);
                out[c * plane + o] = Wn[c];
                out[(m + c) * plane + o] = V / dx;
                out[(2 * m + c) * plane + o] = Y / dy;
                out[(3 * m + c) * plane + o] = 0.5 * (Zx + Zy) / (dx * dy);
            }
            bad |= nonphysical(cfg, 2, Wn);
        }
#undef FH
#undef WX
#undef GH
#undef WY
    free(Fh); free(Wx); free(tst); free(tfl); free(Gt); free(Wyt);
    return bad;
}

double orc_dt2d(const orc_cfg *cfg, int nx, int ny, double dx, double dy,
                double cfl, const double *st)
{
    int m = orc_ncomp(cfg->eq, 2);
    size_t plane = (size_t)nx * ny;
    double smax = 0.0;
    for (size_t o = 0; o < plane; ++o) {
        double W[4];
        for (int c = 0; c < m; ++c) W[c] = st[c * plane + o];
        if (nonphysical(cfg, 2, W)) return -1.0;
        double s = wave_speed(cfg, 2, 0, W) / dx + wave_speed(cfg, 2, 1, W) / dy;
        if (s > smax) smax = s;
    }
    return cfl / smax;
}

int orc_advance2d(const orc_cfg *cfg, int nx, int ny, double dx, double dy,
                  double cfl, double T, long max_steps, double *st, double *t,
                  long *steps)
{
    int m = orc_ncomp(cfg->eq, 2);
    size_t nd = 4 * (size_t)m * nx * ny;
    double *tmp = malloc(sizeof(double) * nd);
    int bad = 0;
    while (*t < T && *steps < max_steps) {
        double dt = orc_dt2d(cfg, nx, ny, dx, dy, cfl, st);
        if (dt < 0) { bad = 1; break; }
        int last = 0;
        if (dt >= T - *t) { dt = T - *t; last = 1; }
        bad = orc_step2d(cfg, nx, ny, dx, dy, dt, st, tmp, NULL);
        memcpy(st, tmp, sizeof(double) * nd);
        *t = last ? T : *t + dt;
        ++*steps;
        if (bad) break;
    }
    free(tmp);
    return bad;
}

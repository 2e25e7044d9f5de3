/*
 * riemann.c -- Euler equations: pressure, flux, Jacobian eigensystem, the HLLC
 * Godunov state and the exact Riemann solver.
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle; see shweno_oracle.h).
 *
 * Equation of state E = p/(gamma-1) + rho|u|^2/2 (sec. 5, eqs. (Euler) and (2d) of the
 * 2D Euler example).  The HLLC solver supplies the leading term of the GRP for
 * the Euler system (sec. 2.1.1); the paper names the solver but not its
 * wave-speed estimates, so the Davis estimates are used (a reading).  The exact
 * solver is not part of the scheme: it provides reference solutions.
 */
#include <math.h>
#include <string.h>
#include "shweno_oracle.h"

int orc_invert(int n, const double *A, double *Ainv);

int orc_ncomp(int eq, int dim)
{
    if (eq == ORC_EULER) return dim == 1 ? 3 : 4;
    return 1;
}

/* primitive variables of a conservative Euler state */
static void euler_prim(double gamma, int dim, const double *W, double *rho,
                       double *u, double *v, double *p)
{
    *rho = W[0];
    *u = W[1] / W[0];
    *v = dim == 2 ? W[2] / W[0] : 0.0;
    double E = W[dim == 2 ? 3 : 2];
    *p = (gamma - 1.0) * (E - 0.5 * (*rho) * ((*u) * (*u) + (*v) * (*v)));
}

void orc_euler_eigen(double gamma, int dim, int dir, const double *W,
                     double *lam, double *R, double *L)
{
    double rho, u, v, p;
    euler_prim(gamma, dim, W, &rho, &u, &v, &p);
    double c = sqrt(gamma * p / rho);
    double E = W[dim == 2 ? 3 : 2];
    double H = (E + p) / rho;
    double q2 = 0.5 * (u * u + v * v);
    if (dim == 1) {
        const double cols[3][3] = {
            {1.0, u - c, H - u * c},
            {1.0, u, q2},
            {1.0, u + c, H + u * c}};
        lam[0] = u - c; lam[1] = u; lam[2] = u + c;
        for (int r = 0; r < 3; ++r)
            for (int s = 0; s < 3; ++s) R[r * 3 + s] = cols[s][r];
        orc_invert(3, R, L);
        return;
    }
    double cols[4][4];
    if (dir == 0) {
        const double t[4][4] = {
            {1.0, u - c, v, H - u * c},
            {1.0, u, v, q2},
            {0.0, 0.0, 1.0, v},
            {1.0, u + c, v, H + u * c}};
        memcpy(cols, t, sizeof t);
        lam[0] = u - c; lam[1] = u; lam[2] = u; lam[3] = u + c;
    } else {
        const double t[4][4] = {
            {1.0, u, v - c, H - v * c},
            {1.0, u, v, q2},
            {0.0, 1.0, 0.0, u},
            {1.0, u, v + c, H + v * c}};
        memcpy(cols, t, sizeof t);
        lam[0] = v - c; lam[1] = v; lam[2] = v; lam[3] = v + c;
    }
    for (int r = 0; r < 4; ++r)
        for (int s = 0; s < 4; ++s) R[r * 4 + s] = cols[s][r];
    orc_invert(4, R, L);
}

/* physical flux in x of a conservative Euler state */
void orc_euler_flux_x(double gamma, int dim, const double *W, double *F)
{
    double rho, u, v, p;
    euler_prim(gamma, dim, W, &rho, &u, &v, &p);
    if (dim == 1) {
        F[0] = W[1];
        F[1] = W[1] * u + p;
        F[2] = (W[2] + p) * u;
    } else {
        F[0] = W[1];
        F[1] = W[1] * u + p;
        F[2] = W[2] * u;
        F[3] = (W[3] + p) * u;
    }
}

void orc_hllc_state(double gamma, int dim, const double *WL, const double *WR,
                    double *Wstar)
{
    const int m = dim == 1 ? 3 : 4;
    double rl, ul, vl, pl, rr, ur, vr, pr;
    euler_prim(gamma, dim, WL, &rl, &ul, &vl, &pl);
    euler_prim(gamma, dim, WR, &rr, &ur, &vr, &pr);
    double cl = sqrt(gamma * pl / rl), cr = sqrt(gamma * pr / rr);
    double SL = fmin(ul - cl, ur - cr);
    double SR = fmax(ul + cl, ur + cr);
    double Ss = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur))
              / (rl * (SL - ul) - rr * (SR - ur));
    const double *WK;
    double rk, uk, vk, pk, SK;
    if (0.0 <= SL) { memcpy(Wstar, WL, m * sizeof(double)); return; }
    if (0.0 > SR) { memcpy(Wstar, WR, m * sizeof(double)); return; }
    if (0.0 <= Ss) { WK = WL; rk = rl; uk = ul; vk = vl; pk = pl; SK = SL; }
    else           { WK = WR; rk = rr; uk = ur; vk = vr; pk = pr; SK = SR; }
    double EK = WK[m - 1];
    double f = rk * (SK - uk) / (SK - Ss);
    Wstar[0] = f;
    Wstar[1] = f * Ss;
    if (dim == 2) Wstar[2] = f * vk;
    Wstar[m - 1] = f * (EK / rk + (Ss - uk) * (Ss + pk / (rk * (SK - uk))));
}

/* HLLE flux and state at x/t = 0 in the normal direction x (not part of the
 * paper's scheme: the first-order flux of the positivity safeguard).  Harten,
 * Lax and van Leer's single intermediate state between wave-speed bounds S_L,
 * S_R from Einfeldt (SIAM J. Numer. Anal. 25, 1988): the smaller and larger of
 * the two sides' acoustic speeds and of the Roe-averaged ones.  Between the
 * bounds, the state is the one the integral form of the conservation law
 * gives over the fan, and the flux the one consistent with it. */
void orc_hlle(double gamma, int dim, const double *WL, const double *WR, double *F,
              double *Wstar)
{
    const int m = dim == 1 ? 3 : 4;
    double rl, ul, vl, pl, rr, ur, vr, pr, FL[4], FR[4];
    euler_prim(gamma, dim, WL, &rl, &ul, &vl, &pl);
    euler_prim(gamma, dim, WR, &rr, &ur, &vr, &pr);
    orc_euler_flux_x(gamma, dim, WL, FL);
    orc_euler_flux_x(gamma, dim, WR, FR);
    double cl = sqrt(gamma * pl / rl), cr = sqrt(gamma * pr / rr);
    /* Roe averages: weights sqrt(rho), enthalpy H = (E + p) / rho */
    double sl = sqrt(rl), sr = sqrt(rr);
    double hl = (WL[m - 1] + pl) / rl, hr = (WR[m - 1] + pr) / rr;
    double ut = (sl * ul + sr * ur) / (sl + sr);
    double vt = (sl * vl + sr * vr) / (sl + sr);
    double ht = (sl * hl + sr * hr) / (sl + sr);
    double ct = sqrt((gamma - 1.0) * (ht - 0.5 * (ut * ut + vt * vt)));
    double SL = fmin(ul - cl, ut - ct);
    double SR = fmax(ur + cr, ut + ct);
    if (0.0 <= SL) {
        memcpy(F, FL, m * sizeof(double));
        memcpy(Wstar, WL, m * sizeof(double));
        return;
    }
    if (SR <= 0.0) {
        memcpy(F, FR, m * sizeof(double));
        memcpy(Wstar, WR, m * sizeof(double));
        return;
    }
    for (int c = 0; c < m; ++c) {
        F[c] = (SR * FL[c] - SL * FR[c] + SL * SR * (WR[c] - WL[c])) / (SR - SL);
        Wstar[c] = (SR * WR[c] - SL * WL[c] - (FR[c] - FL[c])) / (SR - SL);
    }
}

/* ---- exact Riemann solver (Newton on the star-pressure equation) -------- */

static void pressure_fn(double g, double p, double rk, double pk, double ck,
                        double *f, double *fd)
{
    if (p <= pk) {
        double pr = p / pk;
        *f = 2.0 * ck / (g - 1.0) * (pow(pr, (g - 1.0) / (2.0 * g)) - 1.0);
        *fd = 1.0 / (rk * ck) * pow(pr, -(g + 1.0) / (2.0 * g));
    } else {
        double ak = 2.0 / ((g + 1.0) * rk), bk = (g - 1.0) / (g + 1.0) * pk;
        double q = sqrt(ak / (bk + p));
        *f = (p - pk) * q;
        *fd = (1.0 - 0.5 * (p - pk) / (bk + p)) * q;
    }
}

double orc_exact_riemann(double g, double rl, double ul, double pl,
                         double rr, double ur, double pr, double s,
                         double out[3])
{
    double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    /* two-rarefaction starting guess */
    double z = (g - 1.0) / (2.0 * g);
    double p = pow((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) /
                   (cl / pow(pl, z) + cr / pow(pr, z)), 1.0 / z);
    if (!(p > 0.0)) p = 1e-8;
    double fl, fdl, fr, fdr;
    for (int it = 0; it < 200; ++it) {
        pressure_fn(g, p, rl, pl, cl, &fl, &fdl);
        pressure_fn(g, p, rr, pr, cr, &fr, &fdr);
        double pn = p - (fl + fr + ur - ul) / (fdl + fdr);
        if (pn < 1e-14) pn = 1e-14;
        double ch = 2.0 * fabs(pn - p) / (pn + p);
        p = pn;
        if (ch < 1e-15) break;
    }
    pressure_fn(g, p, rl, pl, cl, &fl, &fdl);
    pressure_fn(g, p, rr, pr, cr, &fr, &fdr);
    double us = 0.5 * (ul + ur) + 0.5 * (fr - fl);
    double gm = (g - 1.0) / (g + 1.0);
    if (s <= us) {
        if (p <= pl) {
            double shl = ul - cl;
            if (s <= shl) { out[0] = rl; out[1] = ul; out[2] = pl; return p; }
            double cml = cl * pow(p / pl, z);
            double stl = us - cml;
            if (s > stl) {
                out[0] = rl * pow(p / pl, 1.0 / g); out[1] = us; out[2] = p;
                return p;
            }
            double u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s);
            double c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s));
            out[0] = rl * pow(c / cl, 2.0 / (g - 1.0));
            out[1] = u;
            out[2] = pl * pow(c / cl, 2.0 * g / (g - 1.0));
            return p;
        }
        double pml = p / pl;
        double sl = ul - cl * sqrt((g + 1.0) / (2.0 * g) * pml + z);
        if (s <= sl) { out[0] = rl; out[1] = ul; out[2] = pl; return p; }
        out[0] = rl * (pml + gm) / (pml * gm + 1.0); out[1] = us; out[2] = p;
        return p;
    }
    if (p > pr) {
        double pmr = p / pr;
        double sr = ur + cr * sqrt((g + 1.0) / (2.0 * g) * pmr + z);
        if (s >= sr) { out[0] = rr; out[1] = ur; out[2] = pr; return p; }
        out[0] = rr * (pmr + gm) / (pmr * gm + 1.0); out[1] = us; out[2] = p;
        return p;
    }
    double shr = ur + cr;
    if (s >= shr) { out[0] = rr; out[1] = ur; out[2] = pr; return p; }
    double cmr = cr * pow(p / pr, z);
    double str = us + cmr;
    if (s <= str) {
        out[0] = rr * pow(p / pr, 1.0 / g); out[1] = us; out[2] = p;
        return p;
    }
    double u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s);
    double c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s));
    out[0] = rr * pow(c / cr, 2.0 / (g - 1.0));
    out[1] = u;
    out[2] = pr * pow(c / cr, 2.0 * g / (g - 1.0));
    return p;
}

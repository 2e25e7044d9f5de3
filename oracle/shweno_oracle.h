/*
 * shweno_oracle.h -- plain FP64 CPU oracle of one ADER-SHWENO time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.
 * Only the test-suite, the smoke entry point and the CPU-baseline leg of the
 * benchmark load it.  It shares no source with the GPU path and the GPU path
 * never calls it.
 *
 * It follows Luo, Li, Qiu, Zhu, Chen, "A compact simple HWENO scheme with ADER
 * time discretization for hyperbolic conservation laws I: structured meshes"
 * (arXiv 2304.09724):
 *   finite-volume update                  sec. 2, eq. (cons); sec. 3 (2D form)
 *   GRP at a face, Taylor in time         sec. 2.1, eqs. (grp1d), (tay)
 *   leading term (exact / HLLC)           sec. 2.1.1, eq. (leadingterm)
 *   Lax-Wendroff (Cauchy-Kovalevskaya)    sec. 2.1.2, eq. (ck); sec. 3.1
 *   linearised derivative RPs             sec. 2.1.2, eq. (lineq); sec. 3.1, eq. (lineq2d)
 *   state-expansion flux                  sec. 2.2, eq. (flux); sec. 3.1, eq. (fx2d)
 *   SHWENO reconstruction                 sec. 2.3; sec. 3.2 (dimension by dimension)
 *   derivative averages                   sec. 2.4, eqs. (derave), (tay1d), Remarks 1-2;
 *                                         sec. 3.3, eqs. (derave2d), (taylor2dtime)
 *   algorithm                             sec. 4, Steps 1-5
 * Readings of points the paper leaves open are listed beside each function.
 *
 * State layout (same as the library's public layout, so tests can compare
 * arrays directly): planes [q][m][ny][nx], x fastest, q = 0: cell averages W,
 * 1: averages of W_x (V), and in 2D 2: averages of W_y (Y), 3: averages of
 * W_xy (Z).  Components are conservative: (rho, rho u[, rho v], E).
 */
#ifndef SHWENO_ORACLE_H
#define SHWENO_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_ADVECTION = 0, ORC_BURGERS = 1, ORC_EULER = 2 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_TRANSMISSIVE = 1, ORC_BC_REFLECTIVE = 2 };
enum { ORC_W_NONLINEAR = 0, ORC_W_LINEAR = 1, ORC_W_GATED = 2 };

typedef struct {
    int eq;            /* ORC_ADVECTION / ORC_BURGERS / ORC_EULER */
    int charwise;      /* Euler only: 1 = reconstruct characteristic fields */
    int weights;       /* ORC_W_*: nonlinear, linear, or per-cell flags */
    int bc[4];         /* x-low, x-high, y-low, y-high */
    double gamma;      /* ratio of specific heats (Euler) */
    double adv_a;      /* advection speed in x */
    double adv_b;      /* advection speed in y */
    double eps;        /* regulariser of the nonlinear weights */
    double lin_w[3];   /* linear weights: quartic, left linear, right linear */
    int positivity;    /* Euler: 1 = the positivity safeguard of orc_step1d and
                          orc_step2d (an addition, not in the paper; 0 = the
                          paper's scheme) */
} orc_cfg;

/* number of conservative components of an equation in dimension dim */
int orc_ncomp(int eq, int dim);

/* ---- building blocks (exported for the pins) ---------------------------- */

/* Quartic of the big stencil, as coefficients of xi^0..xi^4 on the centre
 * cell xi in [-1/2,1/2], from averages a[0..2] of cells -1,0,1 and the scaled
 * derivative averages b[0] (cell -1), b[1] (cell +1). */
void orc_big_quartic(const double a[3], const double b[2], double c[5]);

/* Smoothness indicator sum_{k>=1} int_{-1/2}^{1/2} (d^k p / dxi^k)^2 dxi of a
 * quartic given by its coefficients. */
double orc_smoothness(const double c[5]);

/* Nonlinear weights (w[0] quartic, w[1] left linear, w[2] right linear). */
void orc_weights(const orc_cfg *cfg, const double a[3], const double b[2], double w[3]);

/* Reconstruction polynomial from data (a,b) and a given weight set w. */
void orc_combine(const orc_cfg *cfg, const double a[3], const double b[2],
                 const double w[3], double c[5]);

/* Full scalar reconstruction: mode ORC_W_LINEAR returns the big quartic. */
void orc_recon_scalar(const orc_cfg *cfg, int mode, const double a[3],
                      const double b[2], double c[5]);

/* Eigen-decomposition of the Euler flux Jacobian in direction dir (0 = x,
 * 1 = y) at conservative state W (dim = 1: 3 components; dim = 2: 4).
 * R is column-major by eigenvector: R[row*m + s] is component row of r_s.
 * L = R^{-1}, computed numerically.  lam ascending. */
void orc_euler_eigen(double gamma, int dim, int dir, const double *W,
                     double *lam, double *R, double *L);

/* HLLC Godunov state at x/t = 0 (Euler, normal direction x). */
void orc_hllc_state(double gamma, int dim, const double *WL, const double *WR,
                    double *Wstar);

/* HLLE (Einfeldt's wave-speed bounds): flux F and state Wstar at x/t = 0
 * (Euler, normal direction x).  Used only by the positivity safeguard. */
void orc_hlle(double gamma, int dim, const double *WL, const double *WR, double *F,
              double *Wstar);

/* Exact Riemann solution of the 1D Euler equations sampled at x/t = s;
 * out = (rho, u, p).  Returns the star pressure. */
double orc_exact_riemann(double gamma, double rl, double ul, double pl,
                         double rr, double ur, double pr, double s,
                         double out[3]);

/* Cauchy-Kovalevskaya: given w[c][a][b][0] (spatial Taylor coefficients of
 * the interface state, a+b<=4; index ((c*5+a)*5+b)*5+k), fill the time
 * layers k=1..4 from the PDE W_t = -F(W)_x - G(W)_y. */
void orc_ck_fill(const orc_cfg *cfg, int dim, double *w);

/* ---- the time step -------------------------------------------------------- */

/* Largest stable step from the cell averages.  1D: cfl*dx / max(|u|+c);
 * 2D: cfl / max((|u|+c)/dx + (|v|+c)/dy).  Returns <0 if a cell is
 * non-physical. */
double orc_dt1d(const orc_cfg *cfg, int n, double dx, double cfl, const double *state);
double orc_dt2d(const orc_cfg *cfg, int nx, int ny, double dx, double dy,
                double cfl, const double *state);

/* One step of size dt.  flags (may be NULL unless cfg->weights is GATED):
 * one byte per cell, non-zero = full nonlinear reconstruction.  Returns 0,
 * or 1 if the new state has a non-finite value, rho<=0 or p<=0.
 * With cfg->positivity (Euler), the faces of cells whose update would be
 * non-physical take the first-order HLLE flux of the two averages at t_n
 * before the step is judged; see step.c. */
int orc_step1d(const orc_cfg *cfg, int n, double dx, double dt,
               const double *in, double *out, const unsigned char *flags);
int orc_step2d(const orc_cfg *cfg, int nx, int ny, double dx, double dy,
               double dt, const double *in, double *out,
               const unsigned char *flags);

/* Repeated CFL steps until t reaches T (last step clamped to T - t). */
int orc_advance1d(const orc_cfg *cfg, int n, double dx, double cfl, double T,
                  long max_steps, double *state, double *t, long *steps);
int orc_advance2d(const orc_cfg *cfg, int nx, int ny, double dx, double dy,
                  double cfl, double T, long max_steps, double *state,
                  double *t, long *steps);

/* ---- learned gate (not part of the paper's method) ---------------------- */

/* 16 features of cell j of a 1D Euler state (ghosts by cfg's boundary
 * conditions) */
void orc_gate_features1d(const orc_cfg *cfg, int n, double dx, const double *st, int j,
                         double f[16]);
/* 16 features of cell (i, j) of a 2D Euler state along dir (0: x, 1: y):
 * the 1D set on the line through the cell, components (rho, m_n, E) */
void orc_gate_features2d(const orc_cfg *cfg, int nx, int ny, double dx, double dy,
                         const double *st, int i, int j, int dir, double f[16]);
/* 1 if the nonlinear weights of cell j (-1..n: ghosts by the boundary
 * conditions) leave the big stencil below level times its linear weight in
 * some characteristic field */
int orc_gate_label1d(const orc_cfg *cfg, int n, double dx, const double *st, int j,
                     double level);
/* MLP 16-32-32-1: logits of n samples, and mean weighted BCE with gradient */
void orc_mlp_forward(int n, const double *params, const double *X, double *logits);
double orc_mlp_backward(int n, const double *params, const double *X, const double *y,
                        double pos_weight, double *grad);

#ifdef __cplusplus
}
#endif
#endif

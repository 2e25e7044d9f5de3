/*
 * mlp.c -- reference of the learned troubled-cell gate: the cell features,
 * the training labels, and an FP64 multilayer perceptron with its loss
 * gradient.
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle; see shweno_oracle.h).
 *
 * The gate is not part of the paper's method; it decides per cell whether the
 * full nonlinear reconstruction (sec. 2.3) is needed or the linear weights
 * (the big-stencil quartic alone) suffice.
 *
 * Features of a 1D Euler cell j (16, single precision in the GPU code), from
 * exactly the data its reconstruction uses (cells j-1, j, j+1 with the
 * boundary conditions' ghost cells): for each conservative component c, with
 * dl = W_j - W_{j-1}, dr = W_{j+1} - W_j, gm = dx V_{j-1}, gp = dx V_{j+1}
 * and S = |dl| + |dr| + |gm| + |gp|,
 *   f[5c .. 5c+3] = (dl, dr, gm, gp) / S   (0 if S < 1e-30),
 *   f[5c+4]       = log2(S^2 + 1e-12) / 32;
 * and f[15] = u / (|u| + c) at cell j (0 if |u| + c = 0), which sets the
 * characteristic projection.
 *
 * 2D Euler (sec. 3.2): a cell has such a set along x and along y, each from
 * the line of cells through it in that direction, with the components
 * (rho, m_n, E) (m_n the momentum normal to the faces the direction's
 * sweep crosses), the derivative averages in that direction, and u_n with c
 * from the full 2D state.  The gate scores both with the same network and
 * takes the nonlinear weights if either score reaches the threshold.
 *
 * Label of a cell at level L: 1 ("troubled") if the characteristic nonlinear
 * reconstruction of the cell gives the big quartic a weight below L times its
 * linear weight in some field.
 *
 * Network: 16 -> 32 (ReLU) -> 32 (ReLU) -> 1 (logit); parameters in one array
 * W1[32][16], b1[32], W2[32][32], b2[32], w3[32], b3 (1633 values).
 * Loss: weighted binary cross-entropy on sigmoid(logit), mean over samples.
 */
#include <math.h>
#include <string.h>
#include "shweno_oracle.h"

void orc_euler_eigen(double gamma, int dim, int dir, const double *W,
                     double *lam, double *R, double *L);
void orc_cell1d(const orc_cfg *cfg, int n, const double *st, int j, double *W, double *V);
void orc_cell2d(const orc_cfg *cfg, int nx, int ny, const double *st, int i, int j,
                double Q[4][4]);

#define H 32
#define NF 16
#define NPAR (H * NF + H + H * H + H + H + 1)

/* features of cell j of a 1D Euler state */
void orc_gate_features1d(const orc_cfg *cfg, int n, double dx, const double *st, int j,
                         double f[NF])
{
    const int m = 3;
    double W[3][3], V[3][3];
    for (int l = 0; l < 3; ++l) orc_cell1d(cfg, n, st, j - 1 + l, W[l], V[l]);
    for (int c = 0; c < m; ++c) {
        double d[4] = {W[1][c] - W[0][c], W[2][c] - W[1][c], dx * V[0][c], dx * V[2][c]};
        double S = fabs(d[0]) + fabs(d[1]) + fabs(d[2]) + fabs(d[3]);
        for (int k = 0; k < 4; ++k) f[5 * c + k] = S >= 1e-30 ? d[k] / S : 0.0;
        f[5 * c + 4] = log2(S * S + 1e-12) / 32.0;
    }
    double rho = W[1][0], u = W[1][1] / rho;
    double p = (cfg->gamma - 1.0) * (W[1][2] - 0.5 * rho * u * u);
    double a2 = cfg->gamma * p / rho;
    double den = fabs(u) + sqrt(a2 > 0.0 ? a2 : 0.0);
    f[15] = den > 0.0 ? u / den : 0.0;
}

/* the 16 features of one line of three cells: W[l][c], D[l][c] (derivative
 * averages along the line) for l = -1, 0, +1; comp: the three components
 * used; ke: |m|^2 of the centre cell (all momenta) */
static void line_features(double gamma, const double W[3][4], const double D[3][4],
                          const int comp[3], double h, double ke, double f[NF])
{
    for (int k = 0; k < 3; ++k) {
        int c = comp[k];
        double d[4] = {W[1][c] - W[0][c], W[2][c] - W[1][c], h * D[0][c], h * D[2][c]};
        double S = fabs(d[0]) + fabs(d[1]) + fabs(d[2]) + fabs(d[3]);
        for (int q = 0; q < 4; ++q) f[5 * k + q] = S >= 1e-30 ? d[q] / S : 0.0;
        f[5 * k + 4] = log2(S * S + 1e-12) / 32.0;
    }
    double rho = W[1][0], un = W[1][comp[1]] / rho;
    double p = (gamma - 1.0) * (W[1][comp[2]] - 0.5 * ke / rho);
    double a2 = gamma * p / rho;
    double den = fabs(un) + sqrt(a2 > 0.0 ? a2 : 0.0);
    f[15] = den > 0.0 ? un / den : 0.0;
}

/* features of cell (i, j) of a 2D Euler state along direction dir (0: x, 1: y) */
void orc_gate_features2d(const orc_cfg *cfg, int nx, int ny, double dx, double dy,
                         const double *st, int i, int j, int dir, double f[NF])
{
    double Q[3][4][4], W[3][4], D[3][4];
    for (int l = 0; l < 3; ++l) {
        orc_cell2d(cfg, nx, ny, st, dir == 0 ? i - 1 + l : i, dir == 0 ? j : j - 1 + l, Q[l]);
        for (int c = 0; c < 4; ++c) {
            W[l][c] = Q[l][0][c];
            D[l][c] = Q[l][dir == 0 ? 1 : 2][c];
        }
    }
    const int comp[3] = {0, dir == 0 ? 1 : 2, 3};
    double ke = W[1][1] * W[1][1] + W[1][2] * W[1][2];
    line_features(cfg->gamma, W, D, comp, dir == 0 ? dx : dy, ke, f);
}

/* 1 if a characteristic field's big-stencil weight falls below level times
 * its linear weight (data: averages and dx-scaled derivative averages of
 * cells -1, 0, +1 along one direction; dim/dir select the eigenvectors) */
static int troubled_line(const orc_cfg *cfg, int dim, int dir, const double W[3][4],
                         const double B[2][4], double level)
{
    int m = orc_ncomp(cfg->eq, dim);
    double lam[4], R[16], L[16];
    orc_euler_eigen(cfg->gamma, dim, dir, W[1], lam, R, L);
    for (int s = 0; s < m; ++s) {
        double a[3], b[2], w[3];
        for (int l = 0; l < 3; ++l) {
            a[l] = 0.0;
            for (int c = 0; c < m; ++c) a[l] += L[s * m + c] * W[l][c];
        }
        for (int l = 0; l < 2; ++l) {
            b[l] = 0.0;
            for (int c = 0; c < m; ++c) b[l] += L[s * m + c] * B[l][c];
        }
        orc_weights(cfg, a, b, w);
        if (w[0] < level * cfg->lin_w[0]) return 1;
    }
    return 0;
}

int orc_gate_label1d(const orc_cfg *cfg, int n, double dx, const double *st, int j,
                     double level)
{
    double W[3][4], V[3][4], B[2][4];
    for (int l = 0; l < 3; ++l) orc_cell1d(cfg, n, st, j - 1 + l, W[l], V[l]);
    for (int c = 0; c < 3; ++c) {
        B[0][c] = dx * V[0][c];
        B[1][c] = dx * V[2][c];
    }
    return troubled_line(cfg, 1, 0, W, B, level);
}

/* forward pass; h1, h2 (32 each) may be NULL */
double orc_mlp_logit(const double *p, const double x[NF], double *h1, double *h2)
{
    const double *W1 = p, *b1 = W1 + H * NF, *W2 = b1 + H, *b2 = W2 + H * H;
    const double *w3 = b2 + H, *b3 = w3 + H;
    double a1[H], a2[H];
    for (int i = 0; i < H; ++i) {
        double s = b1[i];
        for (int k = 0; k < NF; ++k) s += W1[i * NF + k] * x[k];
        a1[i] = s > 0.0 ? s : 0.0;
    }
    for (int i = 0; i < H; ++i) {
        double s = b2[i];
        for (int k = 0; k < H; ++k) s += W2[i * H + k] * a1[k];
        a2[i] = s > 0.0 ? s : 0.0;
    }
    double z = b3[0];
    for (int k = 0; k < H; ++k) z += w3[k] * a2[k];
    if (h1) memcpy(h1, a1, sizeof a1);
    if (h2) memcpy(h2, a2, sizeof a2);
    return z;
}

/* logits of n samples X[n][NF] */
void orc_mlp_forward(int n, const double *p, const double *X, double *z)
{
    for (int s = 0; s < n; ++s) z[s] = orc_mlp_logit(p, X + s * NF, NULL, NULL);
}

/* mean weighted BCE over n samples and its gradient (grad: NPAR values);
 * y: labels 0/1 as doubles; pos_w: weight of positive samples */
double orc_mlp_backward(int n, const double *p, const double *X, const double *y,
                        double pos_w, double *grad)
{
    const double *W1 = p, *b1 = W1 + H * NF, *W2 = b1 + H, *b2 = W2 + H * H;
    const double *w3 = b2 + H;
    (void)b1; (void)b2;
    memset(grad, 0, NPAR * sizeof(double));
    double *gW1 = grad, *gb1 = gW1 + H * NF, *gW2 = gb1 + H, *gb2 = gW2 + H * H;
    double *gw3 = gb2 + H, *gb3 = gw3 + H;
    double loss = 0.0;
    for (int s = 0; s < n; ++s) {
        const double *x = X + s * NF;
        double h1[H], h2[H];
        double z = orc_mlp_logit(p, x, h1, h2);
        double sig = 1.0 / (1.0 + exp(-z));
        double w = y[s] > 0.5 ? pos_w : 1.0;
        /* loss = -w [y log s + (1-y) log(1-s)], stable form */
        double lz = z > 0 ? z + log1p(exp(-z)) : log1p(exp(z));   /* log(1+e^z) */
        loss += w * (lz - y[s] * z);
        double dz = w * (sig - y[s]) / n;
        gb3[0] += dz;
        double d2[H], d1[H];
        for (int k = 0; k < H; ++k) {
            gw3[k] += dz * h2[k];
            d2[k] = h2[k] > 0.0 ? dz * w3[k] : 0.0;
        }
        for (int i = 0; i < H; ++i) {
            gb2[i] += d2[i];
            for (int k = 0; k < H; ++k) gW2[i * H + k] += d2[i] * h1[k];
        }
        for (int k = 0; k < H; ++k) {
            double s1 = 0.0;
            for (int i = 0; i < H; ++i) s1 += W2[i * H + k] * d2[i];
            d1[k] = h1[k] > 0.0 ? s1 : 0.0;
        }
        for (int i = 0; i < H; ++i) {
            gb1[i] += d1[i];
            for (int k = 0; k < NF; ++k) gW1[i * NF + k] += d1[i] * x[k];
        }
    }
    return loss / n;
}

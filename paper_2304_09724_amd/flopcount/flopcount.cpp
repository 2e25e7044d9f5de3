// flopcount.cpp -- algorithmic FP64 operation count of the sweep arithmetic.
//
// Host program: instantiates the kernels' own templated arithmetic
// (csrc/shw_math.h, csrc/sweep1d_math.h) with an operation-counting real type
// and runs it once on representative data.  Every +, -, *, / and sqrt the
// kernel source performs on state-dependent values is counted once; a fused
// multiply-add counts as two.  Work on per-instance constants (dx, dt and the
// like) is not counted.  Prints one JSON object per path.
#include <cmath>
#include <cstdio>

struct Cnt;
struct Tally { long long add = 0, mul = 0, div = 0, sqrt = 0; };
static Tally g;

struct Cnt {
    double v;
    Cnt() : v(0.0) {}
    Cnt(double x) : v(x) {}
    Cnt &operator+=(Cnt o) { ++g.add; v += o.v; return *this; }
    Cnt &operator-=(Cnt o) { ++g.add; v -= o.v; return *this; }
    Cnt &operator*=(Cnt o) { ++g.mul; v *= o.v; return *this; }
};
static inline Cnt operator+(Cnt a, Cnt b) { ++g.add; return a.v + b.v; }
static inline Cnt operator-(Cnt a, Cnt b) { ++g.add; return a.v - b.v; }
static inline Cnt operator*(Cnt a, Cnt b) { ++g.mul; return a.v * b.v; }
static inline Cnt operator/(Cnt a, Cnt b) { ++g.div; return a.v / b.v; }
static inline Cnt operator+(double a, Cnt b) { ++g.add; return a + b.v; }
static inline Cnt operator-(double a, Cnt b) { ++g.add; return a - b.v; }
static inline Cnt operator*(double a, Cnt b) { ++g.mul; return a * b.v; }
static inline Cnt operator/(double a, Cnt b) { ++g.div; return a / b.v; }
static inline Cnt operator+(Cnt a, double b) { ++g.add; return a.v + b; }
static inline Cnt operator-(Cnt a, double b) { ++g.add; return a.v - b; }
static inline Cnt operator*(Cnt a, double b) { ++g.mul; return a.v * b; }
static inline Cnt operator/(Cnt a, double b) { ++g.div; return a.v / b; }
static inline Cnt operator-(Cnt a) { return -a.v; }
static inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
static inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
static inline bool operator<=(double a, Cnt b) { return a <= b.v; }
static inline bool operator>=(Cnt a, double b) { return a.v >= b; }
static inline bool operator<=(Cnt a, double b) { return a.v <= b; }
static inline bool operator>(Cnt a, double b) { return a.v > b; }
static inline bool operator<(Cnt a, double b) { return a.v < b; }
static inline bool operator>(double a, Cnt b) { return a > b.v; }
static inline Cnt sqrt(Cnt a) { ++g.sqrt; return std::sqrt(a.v); }
static inline Cnt fabs(Cnt a) { return std::fabs(a.v); }
static inline Cnt fmin(Cnt a, Cnt b) { return std::fmin(a.v, b.v); }
static inline Cnt fmax(Cnt a, Cnt b) { return std::fmax(a.v, b.v); }

#include "../csrc/sweep1d_math.h"
#include "../csrc/sweep2d_math.h"

using namespace shw;

static void report(const char *name, const Tally &t, const char *unit)
{
    long long flops = t.add + t.mul + t.div + t.sqrt;
    std::printf("{\"path\": \"%s\", \"unit\": \"%s\", \"flops\": %lld, \"add\": %lld, "
                "\"mul\": %lld, \"div\": %lld, \"sqrt\": %lld}\n",
                name, unit, flops, t.add, t.mul, t.div, t.sqrt);
}

// one 1D Euler cell-update: CFL speed of the cell, reconstruction of the cell,
// the GRP/flux of one face, the update
static void euler1d(bool full, const char *name)
{
    DevParams P{};
    P.gamma = 1.4; P.cfl = 0.9; P.eps = 1e-6;
    P.g1 = 0.994; P.g2 = 0.003; P.g3 = 0.003; P.inv_g1 = 1.0 / 0.994;
    P.charwise = 1;
    P.weights = full ? W_NONLINEAR : W_LINEAR;
    constexpr int M = 3;
    Cnt Wm[M] = {1.0, 0.2, 2.6}, W0[M] = {1.1, 0.3, 2.7}, Wp[M] = {1.2, 0.25, 2.8};
    Cnt Vm[M] = {0.1, 0.05, 0.2}, Vp[M] = {0.12, 0.04, 0.21};
    g = Tally();
    Cnt s = wave_speed<EULER>(W0, P);
    (void)s;
    Cnt lo[5][M], hi[5][M];
    recon_cell<EULER, M>(Wm, W0, Wp, Vm, Vp, 0.01, full, full, P, lo, hi);
    Cnt Fh[M], We[M];
    double js[5];
    jet_scales(100.0, js);
    face1d<EULER, M>(hi, lo, js, 0.004, P, Fh, We);
    Cnt Wn[M], Vn[M];
    update1d<M>(W0, Fh, Fh, We, We, 0.4, 100.0, Wn, Vn);
    report(name, g, "cell-update");
}

// one 2D Euler cell-update: per direction, stage 1 of the cell, and at each
// of the 4 edge nodes stage 2 (5 transverse orders, incl. the node values of
// the stage-1 polynomials), the GRP of one interface node and its
// Gauss-Lobatto flux, then the update; plus the CFL speed of the new average.
static void euler2d(bool full, const char *name)
{
    DevParams P{};
    P.gamma = 1.4; P.cfl = 0.9; P.eps = 1e-6;
    P.g1 = 0.994; P.g2 = 0.003; P.g3 = 0.003; P.inv_g1 = 1.0 / 0.994;
    P.charwise = 1;
    P.weights = full ? W_NONLINEAR : W_LINEAR;
    constexpr int M = 4;
    Cnt W[3][M], V[3][M], Y[3][M], Z[3][M];
    for (int l = 0; l < 3; ++l)
        for (int c = 0; c < M; ++c) {
            W[l][c] = c == 0 ? 1.0 + 0.1 * l : (c == 3 ? 2.6 + 0.1 * l : 0.1 * (c + l));
            V[l][c] = 0.01 * (l + c + 1);
            Y[l][c] = 0.02 * (l - c);
            Z[l][c] = 0.003 * (l + 2 * c);
        }
    const double sc[5] = {1.0, 100.0, 1e4, 1e6, 1e8};
    g = Tally();
    for (int dir = 0; dir < 2; ++dir) {
        Cnt PW[M][5], PV[M][5];
        stage1<M, EULER>(W, V, Y, Z, 0.01, full, full, P, PW, PV);
        for (int gn = 0; gn < 4; ++gn) {
            const double eta = gn == 0 ? -0.5 : gn == 1 ? -LOB_H : gn == 2 ? LOB_H : 0.5;
            CharX<Cnt> Em;
            char_x(W[1], P.gamma, Em);
            Cnt w[M][3], lo[5][M], hi[5][M];
            Cnt JL[15][M], JR[15][M];
            for (int n = 0; n <= 4; ++n) {
                Cnt a0[M], b0[M];
                for (int c = 0; c < M; ++c) {
                    a0[c] = taylor_at(PW[c], eta, n, sc[n]);
                    b0[c] = taylor_at(PV[c], eta, n, sc[n]);
                }
                stage2_order<M, EULER>(n, a0, a0, a0, b0, b0, Em, 0.01, sc, full, full, P, w, lo, hi);
                for (int a = 0; a + n <= 4; ++a)
                    for (int c = 0; c < M; ++c) {
                        JL[jidx(a, n)][c] = hi[a][c];
                        JR[jidx(a, n)][c] = lo[a][c];
                    }
            }
            Cnt wt[M][5], F[M], We[M];
            grp2d<M, EULER>(JL, JR, P, 0.0, 0.0, wt);
            node_flux<M, EULER>(wt, 0.002, P, 0.0, F, We);
            // flux and edge-node accumulation (kernel: Fh += w_g F; dv, corner terms)
            for (int c = 0; c < M; ++c) {
                Cnt acc = LOB_W1 * F[c];
                Cnt dv = LOB_W1 * (We[c] - We[c]);
                (void)acc; (void)dv;
            }
        }
        // update: W -= r (Fu - Fh); Z half: 0.5 (a - b - c + d) * inv
        for (int c = 0; c < M; ++c) {
            Cnt Wn = W[1][c] - 0.3 * (W[0][c] - W[2][c]);
            Cnt zc = 0.5 * (W[0][c] - W[1][c] - W[2][c] + W[0][c]) * 100.0;
            Cnt vn = (W[0][c] + W[1][c]) * 100.0;
            (void)Wn; (void)zc; (void)vn;
        }
    }
    // CFL speed of the new average
    {
        Cnt ir = 1.0 / W[1][0];
        Cnt u = W[1][1] * ir, v = W[1][2] * ir;
        Cnt p = (P.gamma - 1.0) * (W[1][3] - 0.5 * W[1][0] * (u * u + v * v));
        Cnt c = sqrt(P.gamma * p * ir);
        Cnt sp = (fabs(u) + c) * 100.0 + (fabs(v) + c) * 100.0;
        (void)sp;
    }
    report(name, g, "cell-update");
}

int main()
{
    euler1d(true, "euler1d_nonlinear_charwise");
    euler1d(false, "euler1d_linear");
    euler2d(true, "euler2d_nonlinear_charwise");
    euler2d(false, "euler2d_linear");
    return 0;
}

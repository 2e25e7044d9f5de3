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
    P.g1 = 0.994; P.g2 = 0.003; P.g3 = 0.003;
    P.charwise = 1;
    P.weights = full ? W_NONLINEAR : W_LINEAR;
    constexpr int M = 3;
    Cnt Wm[M] = {1.0, 0.2, 2.6}, W0[M] = {1.1, 0.3, 2.7}, Wp[M] = {1.2, 0.25, 2.8};
    Cnt Vm[M] = {0.1, 0.05, 0.2}, Vp[M] = {0.12, 0.04, 0.21};
    g = Tally();
    Cnt s = wave_speed<EULER>(W0, P);
    (void)s;
    Cnt lo[5][M], hi[5][M];
    recon_cell<EULER, M>(Wm, W0, Wp, Vm, Vp, 0.01, full, P, lo, hi);
    Cnt Fh[M], We[M];
    face1d<EULER, M>(hi, lo, 0.004, P, Fh, We);
    Cnt Wn[M], Vn[M];
    update1d<M>(W0, Fh, Fh, We, We, 0.4, 100.0, Wn, Vn);
    report(name, g, "cell-update");
}

int main()
{
    euler1d(true, "euler1d_nonlinear_charwise");
    euler1d(false, "euler1d_linear");
    return 0;
}

// sweep_host.cpp -- host build of the sweep arithmetic for CPU tests.
//
// The kernels' per-point arithmetic is templated on the real type; this file
// instantiates it with R = double on the host, so the tests can check the
// very source the GPU compiles against the oracle without a GPU.  On the host
// the reciprocals and roots are IEEE divisions and square roots (the device
// refines hardware estimates instead); everything else is the same code.
// Test infrastructure: it includes the library's headers, not the oracle's.
#include "../../paper_2304_09724_amd/csrc/sweep1d_math.h"
#include "../../paper_2304_09724_amd/csrc/sweep2d_math.h"

using namespace shw;

static DevParams params(double gamma)
{
    DevParams P{};
    P.gamma = gamma;
    P.charwise = 1;
    P.weights = W_NONLINEAR;
    return P;
}

// 2D Lax-Wendroff series: s[c][a][b] (c < 4, a + b <= 4) the conservative
// spatial Taylor coefficients at the point, wt[c][k] its time coefficients.
extern "C" void host_ck2d_euler(const double *s, double gamma, double *wt)
{
    double S[4][5][5] = {}, W[4][5];
    for (int c = 0; c < 4; ++c)
        for (int a = 0; a < 5; ++a)
            for (int b = 0; a + b < 5; ++b) S[c][a][b] = s[(c * 5 + a) * 5 + b];
    ck2d_euler(S, gamma, W);
    for (int c = 0; c < 4; ++c)
        for (int k = 0; k < 5; ++k) wt[c * 5 + k] = W[c][k];
}

// 1D Lax-Wendroff series: w[c][a] (c < 3) the spatial Taylor coefficients,
// wt[c][k] the time coefficients at the point.
extern "C" void host_ck1d_euler(const double *w, double gamma, double *wt)
{
    double S[3][5][5] = {};
    for (int c = 0; c < 3; ++c)
        for (int a = 0; a < 5; ++a) S[c][a][0] = w[c * 5 + a];
    const DevParams P = params(gamma);
    ck1d<EULER, 3>(S, P);
    for (int c = 0; c < 3; ++c)
        for (int k = 0; k < 5; ++k) wt[c * 5 + k] = S[c][0][k];
}

// The whole 2D GRP at one interface point (normal s): jl, jr [15][4] the
// two sides' series coefficients d^{a+n}W/ds^a dt^n / (a! n!) at index
// jidx(a, n); wt[c][k] the time coefficients.
extern "C" void host_grp2d_euler(const double *jl, const double *jr, double gamma, double *wt)
{
    double JL[15][4], JR[15][4], W[4][5];
    for (int i = 0; i < 15; ++i)
        for (int c = 0; c < 4; ++c) {
            JL[i][c] = jl[i * 4 + c];
            JR[i][c] = jr[i * 4 + c];
        }
    const DevParams P = params(gamma);
    grp2d<4, EULER>(JL, JR, P, 0.0, 0.0, W);
    for (int c = 0; c < 4; ++c)
        for (int k = 0; k < 5; ++k) wt[c * 5 + k] = W[c][k];
}

extern "C" int host_jidx(int a, int n) { return jidx(a, n); }

// gate_math.h -- the learned troubled-cell gate on the device: cell features,
// training labels, and the 8-32-32-1 network evaluated by one wave with
// BF16 matrix-core instructions (FP32 accumulation).
//
// The gate is an addition to the paper's method: a cell it passes as smooth
// takes the linear weights (the big-stencil quartic alone, sec. 2.3) instead
// of the nonlinear SHWENO reconstruction; everything else stays FP64.
#pragma once

#include "shw_math.h"

namespace shw {

constexpr int GATE_H = 32;
constexpr int GATE_NF = 8;
constexpr int GATE_NPAR = GATE_H * GATE_NF + GATE_H + GATE_H * GATE_H + GATE_H + GATE_H + 1;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Network parameters laid out per lane of a wave exactly as the matrix
// instructions consume them (built on the host from the FP32 parameters):
// lane l holds the A-operand slices of W1 and W2 and the bias/output-weight
// values of the 16 accumulator rows it owns.
struct GateLane {
    bf16x4 w1;          // W1[l%32][4(l/32) + e]
    bf16x4 w2[4];       // W2[l%32][8q + 4(l/32) + e], K-chunk q
    float b1[16];       // b1[row(v)]
    float b2[16];       // b2[row(v)]
    float w3[16];       // w3[row(v)]
    float b3;
    float pad[3];
};

// accumulator row of item v held by lane l (32x32x8 layout)
SHW_HD constexpr int mfma_row(int lane, int v) { return 8 * (v / 4) + 4 * (lane / 32) + (v % 4); }

__device__ __forceinline__ short f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);         // round to nearest even
    return (short)(u >> 16);
}

// Feature transform: log2(x + 1e-12) / 32.
__device__ __forceinline__ float gate_logfeat(double x) { return log2f((float)(x + 1e-12)) * (1.0f / 32.0f); }

// Features of one 1D Euler cell from its own and its neighbours' averages and
// its derivative average (density and energy: jumps to both sides, their
// difference, dx V).
__device__ __forceinline__ void gate_features1d(const double Wm[3], const double W0[3],
                                                const double Wp[3], const double V0[3],
                                                double dx, float f[8])
{
    const int qs[2] = {0, 2};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int c = qs[k];
        const double dl = W0[c] - Wm[c], dr = Wp[c] - W0[c], b = dx * V0[c];
        f[4 * k + 0] = gate_logfeat(dl * dl);
        f[4 * k + 1] = gate_logfeat(dr * dr);
        f[4 * k + 2] = gate_logfeat((dr - dl) * (dr - dl));
        f[4 * k + 3] = gate_logfeat(b * b);
    }
}

// Training label of one 1D Euler cell: 1 if, in the characteristic
// reconstruction of the cell, some field gives the big quartic less than 0.95
// of its linear weight.
template <int M>
__device__ __forceinline__ int gate_label1d(const double Wm[M], const double W0[M],
                                            const double Wp[M], const double Vm[M],
                                            const double Vp[M], double dx, const DevParams &P)
{
    double R[M][M], L[M][M], lam[M];
    euler_eigen<1, 0>(W0, P.gamma, R, L, lam);
    int bad = 0;
#pragma unroll
    for (int s = 0; s < M; ++s) {
        double am = 0.0, a0 = 0.0, ap = 0.0, bm = 0.0, bp = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            am += L[s][c] * Wm[c];
            a0 += L[s][c] * W0[c];
            ap += L[s][c] * Wp[c];
            bm += L[s][c] * Vm[c];
            bp += L[s][c] * Vp[c];
        }
        double q[5], w[3];
        big_quartic(am, a0, ap, dx * bm, dx * bp, q);
        nonlinear_weights(q, am, a0, ap, P, w);
        bad |= w[0] < 0.95 * P.g1;
    }
    return bad;
}

// Logit of the cell held by each lane (lane = cell, its 8 features in f).
// Must be called by all 64 lanes of a wave together.  Two passes of 32
// cells: H1^T = W1 X^T (one 32x32x8 product), H2^T = W2 H1^T (four, K = 32),
// logit = w3 . H2 + b3 (lane sums over its 16 rows, then with lane l^32).
// The accumulator layout of layer 1 is the B-operand layout of layer 2, so
// no data moves between the layers.
__device__ __forceinline__ float gate_wave_logit(const float f[8], const GateLane &G)
{
    const int lane = threadIdx.x % 64;
    const int half = lane / 32;
    float out = 0.0f;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const int src = 32 * pass + (lane % 32);
        bf16x4 xb;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float lo = __shfl(f[e], src, 64);
            const float hi = __shfl(f[e + 4], src, 64);
            xb[e] = f2bf(half ? hi : lo);
        }
        f32x16 acc;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = G.b1[v];
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(G.w1, xb, acc, 0, 0, 0);
        f32x16 acc2;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc2[v] = G.b2[v];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bf16x4 hb;
#pragma unroll
            for (int e = 0; e < 4; ++e) hb[e] = f2bf(fmaxf(acc[4 * q + e], 0.0f));
            acc2 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(G.w2[q], hb, acc2, 0, 0, 0);
        }
        float s = 0.0f;
#pragma unroll
        for (int v = 0; v < 16; ++v) s += G.w3[v] * fmaxf(acc2[v], 0.0f);
        s += __shfl_xor(s, 32, 64);
        if (pass == half) out = s + G.b3;
    }
    return out;
}

} // namespace shw

// gate_math.h -- the learned troubled-cell gate on the device: cell features,
// training labels, and the 16-32-32-1 network evaluated by one wave with
// BF16 matrix-core instructions (FP32 accumulation).
//
// The gate is an addition to the paper's method: a cell it passes as smooth
// takes the linear weights (the big-stencil quartic alone, sec. 2.3) instead
// of the nonlinear SHWENO reconstruction; everything else stays FP64.
#pragma once

#include "shw_math.h"

namespace shw {

constexpr int GATE_H = 32;
constexpr int GATE_NF = 16;
constexpr int GATE_NPAR = GATE_H * GATE_NF + GATE_H + GATE_H * GATE_H + GATE_H + GATE_H + 1;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Network parameters laid out per lane of a wave exactly as the 32x32x16
// BF16 matrix instruction consumes them (operand A: lane l holds row l%32,
// k = 8(l/32) + e; accumulator item v of lane l is row
// 8(v/4) + 4(l/32) + v%4, column l%32), built on the host from the FP32
// parameters.  BF16 pairs are stored as 32-bit words (element 2i in the low
// half).  256 bytes per lane.
struct GateLane {
    u32x4 w1;           // W1[l%32][8(l/32) + e]
    u32x4 w2[2];        // W2[l%32][gate_hidden(q, l/32, e)], K-chunk q
    float b1[16];       // b1[row(v)]
    float b2[16];       // b2[row(v)]
    float w3[16];       // w3[row(v)]
    float b3;
    float pad[3];
};

static_assert(sizeof(GateLane) == 16 * sizeof(u32x4), "GateLane is 16 words of 16 bytes");

// The LDS copy of a packed network is transposed to [16-byte word][lane]:
// the lanes of a wave then read 1 KB of consecutive bytes per word, without
// bank conflicts (the per-lane structs sit 256 bytes apart, all on the same
// banks).
constexpr int GATE_LDS_WORDS = 16 * 64;

__device__ __forceinline__ void gate_to_lds(const GateLane *g, u32x4 *lds, int tid, int nthreads)
{
    const u32x4 *src = reinterpret_cast<const u32x4 *>(g);
    for (int i = tid; i < GATE_LDS_WORDS; i += nthreads) {
        const int lane = i % 64, word = i / 64;
        lds[i] = src[lane * 16 + word];
    }
}

__device__ __forceinline__ GateLane gate_lane_lds(const u32x4 *lds, int lane)
{
    GateLane G;
    u32x4 *dst = reinterpret_cast<u32x4 *>(&G);
#pragma unroll
    for (int w = 0; w < 16; ++w) dst[w] = lds[w * 64 + lane];
    return G;
}

// accumulator row of item v held by lane l (32x32 output layout)
SHW_HD constexpr int mfma_row(int lane, int v) { return 8 * (v / 4) + 4 * (lane / 32) + (v % 4); }

// The first hidden layer's accumulators feed the second layer's B operand
// without moving: in K-chunk q, element e of a lane in half h is its
// accumulator item 8q + e, i.e. hidden unit mfma_row(32h, 8q + e).  W2's
// columns are packed in the same order.
SHW_HD constexpr int gate_hidden(int q, int h, int e) { return mfma_row(32 * h, 8 * q + e); }

// value of the partner lane l ^ 32 (one swap of the two half-waves)
__device__ __forceinline__ unsigned half_swap(unsigned x)
{
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (threadIdx.x % 64) < 32 ? r[1] : r[0];
}

__device__ __forceinline__ bf16x8 to_bf16(const float *x)
{
    const f32x8 v = {x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7]};
    return __builtin_convertvector(v, bf16x8);      // round to nearest even
}

// Features of one Euler cell along one direction, from exactly the data its
// reconstruction in that direction reads (sec. 2.3; in 2D, sec. 3.2, the
// averages of the line's cells j-1, j, j+1 and the derivative averages of
// j-1, j+1).  Arrays hold the conservative components in the direction's
// frame: M = 3 (rho, m, E) in 1D, M = 4 (rho, m_n, m_t, E) in 2D; the tangential
// momentum, which the 1D network never saw, is left out.  Per component c of
// (rho, m_n, E), with dl, dr the jumps of the averages, gm, gp the
// neighbours' derivative averages times dx and S = |dl| + |dr| + |gm| + |gp|:
// the signed shape (dl, dr, gm, gp) / S (zero if S < 1e-30) and
// log2(S^2 + 1e-12) / 32 (the size against the weights' regulariser); then
// u_n / (|u_n| + c) of the cell, which sets the characteristic projection.
// The differences are formed in FP64, the rest in FP32.
template <int M>
__device__ __forceinline__ void gate_features(const double Wm[M], const double W0[M],
                                              const double Wp[M], const double Vm[M],
                                              const double Vp[M], double dx, double gamma,
                                              float f[GATE_NF])
{
    static_assert(M == 3 || M == 4, "Euler in 1D or 2D");
    const int comp[3] = {0, 1, M - 1};
#pragma unroll
    for (int k3 = 0; k3 < 3; ++k3) {
        const int c = comp[k3];
        const float d[4] = {(float)(W0[c] - Wm[c]), (float)(Wp[c] - W0[c]), (float)(dx * Vm[c]),
                            (float)(dx * Vp[c])};
        const float S = fabsf(d[0]) + fabsf(d[1]) + fabsf(d[2]) + fabsf(d[3]);
        const float iS = S >= 1e-30f ? __builtin_amdgcn_rcpf(S) : 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) f[5 * k3 + k] = d[k] * iS;
        f[5 * k3 + 4] = log2f(S * S + 1e-12f) * (1.0f / 32.0f);
    }
    const float rho = (float)W0[0], E = (float)W0[M - 1];
    const float irho = __builtin_amdgcn_rcpf(rho);
    float ke = 0.0f;
#pragma unroll
    for (int c = 1; c < M - 1; ++c) ke += (float)W0[c] * (float)W0[c];
    const float u = (float)W0[1] * irho;
    const float p = (float)(gamma - 1.0) * (E - 0.5f * ke * irho);
    const float a2 = (float)gamma * p * irho;
    const float den = fabsf(u) + sqrtf(fmaxf(a2, 0.0f));
    f[15] = den > 0.0f ? u * __builtin_amdgcn_rcpf(den) : 0.0f;
}

__device__ __forceinline__ void gate_features1d(const double Wm[3], const double W0[3],
                                                const double Wp[3], const double Vm[3],
                                                const double Vp[3], double dx, double gamma,
                                                float f[GATE_NF])
{
    gate_features<3>(Wm, W0, Wp, Vm, Vp, dx, gamma, f);
}

// Training label of one 1D Euler cell at level L: 1 if, in the cell's
// characteristic reconstruction, some field gives the big quartic less than
// L times its linear weight.
template <int M>
__device__ __forceinline__ int gate_label1d(const double Wm[M], const double W0[M],
                                            const double Wp[M], const double Vm[M],
                                            const double Vp[M], double dx, const DevParams &P,
                                            double level)
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
        bad |= w[0] < level * P.g1;
    }
    return bad;
}

// Logit of the cell held by each lane (lane = cell, its features in f).
// Must be called by all 64 lanes of a wave together.  Two passes of 32
// cells (samples are the B-operand columns): H1^T = W1 X^T (one 32x32x16
// product), H2^T = W2 H1^T (two, K = 32), logit = w3 . H2 + b3 (a lane sums
// its 16 rows, then adds its partner half's).  Operand B of the first layer
// needs, in half h, features 8h..8h+7 of the pass's cells: one half-wave swap
// brings each lane the half its partner holds.
__device__ __forceinline__ float gate_wave_logit(const float f[GATE_NF], const GateLane &G)
{
    const bool lo = (threadIdx.x % 64) < 32;
    const bf16x8 xlo = to_bf16(f), xhi = to_bf16(f + 8);
    u32x4 send = __builtin_bit_cast(u32x4, lo ? xhi : xlo), recv;
#pragma unroll
    for (int i = 0; i < 4; ++i) recv[i] = half_swap(send[i]);
    const bf16x8 got = __builtin_bit_cast(bf16x8, recv);
    const bf16x8 w1 = __builtin_bit_cast(bf16x8, G.w1);
    float out = 0.0f;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        // lanes < 32 hold k = 0..7, lanes >= 32 k = 8..15 of cell 32 pass + l % 32
        const bf16x8 xb = pass == 0 ? (lo ? xlo : got) : (lo ? got : xhi);
        f32x16 acc;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = G.b1[v];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, xb, acc, 0, 0, 0);
        f32x16 acc2;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc2[v] = G.b2[v];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            float h[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) h[e] = fmaxf(acc[8 * q + e], 0.0f);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, G.w2[q]),
                                                          to_bf16(h), acc2, 0, 0, 0);
        }
        float s = 0.0f;
#pragma unroll
        for (int v = 0; v < 16; ++v) s += G.w3[v] * fmaxf(acc2[v], 0.0f);
        s += __uint_as_float(half_swap(__float_as_uint(s)));
        if (pass == (lo ? 0 : 1)) out = s + G.b3;
    }
    return out;
}

} // namespace shw

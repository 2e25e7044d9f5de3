// gate.hip -- kernels of the learned troubled-cell gate: training data from
// the method's own quantities (features and labels of every cell of a 1D
// batch), BF16 matrix-core inference, and FP32 training (forward + backward
// with block reductions, then Adam).
#include "gate_math.h"
#include "shw_kernels.h"
#include "sweep1d_math.h"

namespace shw {

namespace {

constexpr int TB = 128;          // samples per training block

// features and label of every cell (grid: cells x instances)
__global__ void __launch_bounds__(256) gate_data1d_kernel(const Inst1D *inst, const double *state,
                                                          DevParams P, double level, float *feat,
                                                          uint8_t *label)
{
    constexpr int M = 3;
    const Inst1D d = inst[blockIdx.y];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d.n) return;
    const double *src = state + d.off;
    // three separately named cells, as in the sweep (a [3][M] array here was
    // packed into one vector whose ghost-branch merge gave wrong derivative
    // averages at the first cell)
    double Wm[M], Vm[M], W0[M], V0[M], Wp[M], Vp[M];
    load_cell<EULER, M>(src, d.n, j - 1, d.bc_lo, d.bc_hi, Wm, Vm);
    load_cell<EULER, M>(src, d.n, j, d.bc_lo, d.bc_hi, W0, V0);
    load_cell<EULER, M>(src, d.n, j + 1, d.bc_lo, d.bc_hi, Wp, Vp);
    float f[GATE_NF];
    gate_features1d(Wm, W0, Wp, Vm, Vp, d.dx, P.gamma, f);
    const long long o = d.cell_off + j;
#pragma unroll
    for (int k = 0; k < GATE_NF; ++k) feat[o * GATE_NF + k] = f[k];
    label[o] = (uint8_t)gate_label1d<M>(Wm, W0, Wp, Vm, Vp, d.dx, P, level);
}

// logits of n samples (one wave per 64 samples; all lanes take part)
__global__ void __launch_bounds__(256) mlp_logits_kernel(const float *X, int n, const GateLane *G,
                                                         float *logits)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % 64;
    float f[GATE_NF];
#pragma unroll
    for (int k = 0; k < GATE_NF; ++k) f[k] = i < n ? X[(long long)i * GATE_NF + k] : 0.0f;
    const GateLane g = G[lane];
    const float z = gate_wave_logit(f, g);
    if (i < n) logits[i] = z;
}

__global__ void zero_f32_kernel(float *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// Gradient of the mean weighted binary cross-entropy of sigmoid(logit) over
// n samples, accumulated into grad (FP32); loss into *loss.  One thread per
// sample for the forward and the per-sample deltas; the parameter gradients
// are sums over the block's samples formed from LDS, then one atomic add per
// parameter per block.
__global__ void __launch_bounds__(TB) mlp_grad_kernel(const float *X, const float *y, int n,
                                                      const float *p, float pos_w, float *grad,
                                                      float *loss)
{
    __shared__ float sx[TB][GATE_NF];
    __shared__ float sh1[TB][GATE_H + 1];
    __shared__ float sd1[TB][GATE_H + 1];
    __shared__ float sd2[TB][GATE_H + 1];
    __shared__ float sh2[TB][GATE_H + 1];
    __shared__ float sdz[TB];
    const float *W1 = p, *b1 = W1 + GATE_H * GATE_NF, *W2 = b1 + GATE_H, *b2 = W2 + GATE_H * GATE_H;
    const float *w3 = b2 + GATE_H, *b3 = w3 + GATE_H;
    const int t = threadIdx.x;
    const long long i = (long long)blockIdx.x * TB + t;
    const bool ok = i < n;
    float x[GATE_NF];
#pragma unroll
    for (int k = 0; k < GATE_NF; ++k) x[k] = ok ? X[i * GATE_NF + k] : 0.0f;
    float h1[GATE_H], h2[GATE_H];
#pragma unroll
    for (int r = 0; r < GATE_H; ++r) {
        float s = b1[r];
#pragma unroll
        for (int k = 0; k < GATE_NF; ++k) s += W1[r * GATE_NF + k] * x[k];
        h1[r] = fmaxf(s, 0.0f);
    }
    float z = b3[0];
#pragma unroll
    for (int r = 0; r < GATE_H; ++r) {
        float s = b2[r];
#pragma unroll
        for (int k = 0; k < GATE_H; ++k) s += W2[r * GATE_H + k] * h1[k];
        h2[r] = fmaxf(s, 0.0f);
        z += w3[r] * h2[r];
    }
    const float yy = ok ? y[i] : 0.0f;
    const float wgt = yy > 0.5f ? pos_w : 1.0f;
    const float sig = 1.0f / (1.0f + expf(-z));
    const float lz = z > 0.0f ? z + log1pf(expf(-z)) : log1pf(expf(z));
    const float dz = ok ? wgt * (sig - yy) / (float)n : 0.0f;
    const float li = ok ? wgt * (lz - yy * z) / (float)n : 0.0f;
    float d2[GATE_H];
#pragma unroll
    for (int r = 0; r < GATE_H; ++r) d2[r] = h2[r] > 0.0f ? dz * w3[r] : 0.0f;
#pragma unroll
    for (int k = 0; k < GATE_H; ++k) {
        float s = 0.0f;
#pragma unroll
        for (int r = 0; r < GATE_H; ++r) s += W2[r * GATE_H + k] * d2[r];
        sd1[t][k] = h1[k] > 0.0f ? s : 0.0f;
        sh1[t][k] = h1[k];
        sh2[t][k] = h2[k];
        sd2[t][k] = d2[k];
    }
#pragma unroll
    for (int k = 0; k < GATE_NF; ++k) sx[t][k] = x[k];
    sdz[t] = dz;
    __syncthreads();
    float *gW1 = grad, *gb1 = gW1 + GATE_H * GATE_NF, *gW2 = gb1 + GATE_H, *gb2 = gW2 + GATE_H * GATE_H;
    float *gw3 = gb2 + GATE_H, *gb3 = gw3 + GATE_H;
    // dW2[r][k] = sum_s d2[s][r] h1[s][k]: 1024 entries, 8 per thread
    for (int e = t; e < GATE_H * GATE_H; e += TB) {
        const int r = e / GATE_H, k = e % GATE_H;
        float s = 0.0f;
        for (int q = 0; q < TB; ++q) s += sd2[q][r] * sh1[q][k];
        atomicAdd(&gW2[e], s);
    }
    for (int e = t; e < GATE_H * GATE_NF; e += TB) {
        const int r = e / GATE_NF, k = e % GATE_NF;
        float s = 0.0f;
        for (int q = 0; q < TB; ++q) s += sd1[q][r] * sx[q][k];
        atomicAdd(&gW1[e], s);
    }
    if (t < GATE_H) {
        float s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
        for (int q = 0; q < TB; ++q) {
            s1 += sd1[q][t];
            s2 += sd2[q][t];
            s3 += sdz[q] * sh2[q][t];
        }
        atomicAdd(&gb1[t], s1);
        atomicAdd(&gb2[t], s2);
        atomicAdd(&gw3[t], s3);
    }
    // loss and gb3: wave sums, one atomic per wave
    float a = li, bsum = dz;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        bsum += __shfl_xor(bsum, o, 64);
    }
    if (t % 64 == 0) {
        atomicAdd(loss, a);
        atomicAdd(gb3, bsum);
    }
}

// Adam step (FP32 master parameters), t = step number from 1
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int n, int t, float lr,
                            float beta1, float beta2, float eps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(beta1, (float)t));
    const float vh = vi / (1.0f - powf(beta2, (float)t));
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

} // namespace

hipError_t launch_gate_data1d(const Inst1D *inst, int n_inst, int max_n, const double *state,
                              const DevParams &P, double level, float *feat, uint8_t *label,
                              hipStream_t st)
{
    dim3 grid((max_n + 255) / 256, n_inst);
    gate_data1d_kernel<<<grid, 256, 0, st>>>(inst, state, P, level, feat, label);
    return hipGetLastError();
}

hipError_t launch_mlp_logits(const float *X, int n, const GateLane *G, float *logits,
                             hipStream_t st)
{
    mlp_logits_kernel<<<(n + 255) / 256, 256, 0, st>>>(X, n, G, logits);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *X, const float *y, int n, const float *p, float pos_w,
                           float *grad, float *loss, hipStream_t st)
{
    zero_f32_kernel<<<(GATE_NPAR + 255) / 256, 256, 0, st>>>(grad, GATE_NPAR);
    zero_f32_kernel<<<1, 1, 0, st>>>(loss, 1);
    mlp_grad_kernel<<<(n + TB - 1) / TB, TB, 0, st>>>(X, y, n, p, pos_w, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int t, float lr,
                       hipStream_t st)
{
    adam_kernel<<<(GATE_NPAR + 255) / 256, 256, 0, st>>>(p, g, m, v, GATE_NPAR, t, lr, 0.9f,
                                                         0.999f, 1e-8f);
    return hipGetLastError();
}

} // namespace shw

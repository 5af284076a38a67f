// Learned Verlet-buffer predictor: hand-written training and inference
// kernels for an 8-64-64-1 multilayer perceptron (not part of the paper; it
// learns the buffer the paper's drift criterion needs, Sec. 5, from exact
// missed-pair recounts).
//
// x (8 raw features) -> normalised to [-1, 1] with the model's feature ranges
//   -> h1 = tanh(W1 x + b1) -> h2 = tanh(W2 h1 + b2) -> y = softplus(w3.h2 + b3)
// Loss: mean squared error over the batch; optimiser: Adam with bias
// correction (beta1 0.9, beta2 0.999, eps 1e-8).  Flat parameter order:
// W1 (64x8 row-major), b1, W2 (64x64 row-major), b2, w3, b3 -- 4801 floats.
//
// Mapping: a workgroup of four wavefronts; lane j of a wavefront is hidden
// unit j of both layers and keeps its rows of W1 and W2 (and their gradient
// accumulators) in registers.  Hidden activations and the layer-2 deltas are
// broadcast through LDS; the column access W2^T delta2 reads a padded LDS
// copy of W2 without bank conflicts.
#include "internal.h"

namespace {

constexpr int NF = 8, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NF, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;
static_assert(NPARAM == 4801, "parameter count");

struct MlpArgs {
    float *params, *m, *v;
    int *step;
    const float *lo, *hi;
    const float *X, *y;
    int batch;
    float lr;
    float *loss;
    float *grad_out;   // non-null: write the batch gradient, do not update
    float *y_out;      // inference output
};

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline float wsum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline float softplus(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }

__device__ inline float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

__global__ __launch_bounds__(256) void k_mlp_step(MlpArgs a) {
    __shared__ float w2s[NH * (NH + 1)];
    __shared__ float h1s[4][NH], d2s[4][NH];
    __shared__ float gacc[NPARAM + 1];   // gradient, then the loss sum
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int i = tid; i < NH * NH; i += 256) w2s[(i / NH) * (NH + 1) + i % NH] = a.params[OFF_W2 + i];
    for (int i = tid; i <= NPARAM; i += 256) gacc[i] = 0.0f;
    __syncthreads();
    float w1[NF], gw1[NF], w2[NH], gw2[NH], lo[NF], sc[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        w1[i] = a.params[OFF_W1 + lane * NF + i];
        gw1[i] = 0.0f;
        lo[i] = a.lo[i];
        sc[i] = 2.0f / (a.hi[i] - a.lo[i]);
    }
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        w2[i] = w2s[lane * (NH + 1) + i];
        gw2[i] = 0.0f;
    }
    const float b1 = a.params[OFF_B1 + lane], b2 = a.params[OFF_B2 + lane], w3 = a.params[OFF_W3 + lane];
    const float b3 = a.params[OFF_B3];
    float gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f, gb3 = 0.0f, lsum = 0.0f;
    const float inv_b = 2.0f / (float)a.batch;
    for (int s = w; s < a.batch; s += 4) {
        float x[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i) x[i] = (a.X[s * NF + i] - lo[i]) * sc[i] - 1.0f;
        float z1 = b1;
#pragma unroll
        for (int i = 0; i < NF; ++i) z1 = fmaf(w1[i], x[i], z1);
        const float h1 = tanhf(z1);
        h1s[w][lane] = h1;
        wave_sync_lds();
        float z2 = b2;
#pragma unroll
        for (int i = 0; i < NH; ++i) z2 = fmaf(w2[i], h1s[w][i], z2);
        const float h2 = tanhf(z2);
        const float z3 = wsum(w3 * h2) + b3;
        const float r = softplus(z3) - a.y[s];
        lsum += r * r;
        const float d3 = inv_b * r * sigmoid(z3);
        gw3 = fmaf(d3, h2, gw3);
        gb3 += d3;
        const float d2 = d3 * w3 * (1.0f - h2 * h2);
        gb2 += d2;
#pragma unroll
        for (int i = 0; i < NH; ++i) gw2[i] = fmaf(d2, h1s[w][i], gw2[i]);
        d2s[w][lane] = d2;
        wave_sync_lds();
        float s1 = 0.0f;
#pragma unroll 16
        for (int k = 0; k < NH; ++k) s1 = fmaf(w2s[k * (NH + 1) + lane], d2s[w][k], s1);
        const float d1 = (1.0f - h1 * h1) * s1;
        gb1 += d1;
#pragma unroll
        for (int i = 0; i < NF; ++i) gw1[i] = fmaf(d1, x[i], gw1[i]);
        wave_sync_lds();   // before the next sample overwrites h1s / d2s
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) atomicAdd(&gacc[OFF_W1 + lane * NF + i], gw1[i]);
    atomicAdd(&gacc[OFF_B1 + lane], gb1);
#pragma unroll
    for (int i = 0; i < NH; ++i) atomicAdd(&gacc[OFF_W2 + lane * NH + i], gw2[i]);
    atomicAdd(&gacc[OFF_B2 + lane], gb2);
    atomicAdd(&gacc[OFF_W3 + lane], gw3);
    if (lane == 0) {
        atomicAdd(&gacc[OFF_B3], gb3);
        atomicAdd(&gacc[NPARAM], lsum);
    }
    __syncthreads();
    if (a.loss && tid == 0) *a.loss = gacc[NPARAM] / (float)a.batch;
    if (a.grad_out) {
        for (int i = tid; i < NPARAM; i += 256) a.grad_out[i] = gacc[i];
        return;
    }
    const int t = *a.step + 1;
    const float c1 = 1.0f / (1.0f - powf(0.9f, (float)t)), c2 = 1.0f / (1.0f - powf(0.999f, (float)t));
    for (int i = tid; i < NPARAM; i += 256) {
        const float g = gacc[i];
        const float m = 0.9f * a.m[i] + 0.1f * g;
        const float v = 0.999f * a.v[i] + 0.001f * g * g;
        a.m[i] = m;
        a.v[i] = v;
        a.params[i] -= a.lr * (m * c1) / (sqrtf(v * c2) + 1e-8f);
    }
    __syncthreads();
    if (tid == 0) *a.step = t;
}

// Inference: each wavefront evaluates samples s = wave, wave + waves, ...
__global__ __launch_bounds__(256) void k_mlp_infer(MlpArgs a) {
    __shared__ float h1s[4][NH];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    float w1[NF], w2[NH], lo[NF], sc[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        w1[i] = a.params[OFF_W1 + lane * NF + i];
        lo[i] = a.lo[i];
        sc[i] = 2.0f / (a.hi[i] - a.lo[i]);
    }
#pragma unroll
    for (int i = 0; i < NH; ++i) w2[i] = a.params[OFF_W2 + lane * NH + i];
    const float b1 = a.params[OFF_B1 + lane], b2 = a.params[OFF_B2 + lane], w3 = a.params[OFF_W3 + lane];
    const float b3 = a.params[OFF_B3];
    for (int s = blockIdx.x * 4 + w; s < a.batch; s += gridDim.x * 4) {
        float z1 = b1;
#pragma unroll
        for (int i = 0; i < NF; ++i) z1 = fmaf(w1[i], (a.X[s * NF + i] - lo[i]) * sc[i] - 1.0f, z1);
        h1s[w][lane] = tanhf(z1);
        wave_sync_lds();
        float z2 = b2;
#pragma unroll
        for (int i = 0; i < NH; ++i) z2 = fmaf(w2[i], h1s[w][i], z2);
        const float z3 = wsum(w3 * tanhf(z2)) + b3;
        if (lane == 0) a.y_out[s] = softplus(z3);
        wave_sync_lds();
    }
}

}  // namespace

namespace mxn {

int launch_mlp_step(nb_ctx *ctx, nb_mlp *mlp, const float *X, const float *y, int batch, float lr, float *loss,
                    float *grad_out) {
    MlpArgs a{};
    a.params = (float *)mlp->params.p;
    a.m = (float *)mlp->m.p;
    a.v = (float *)mlp->v.p;
    a.step = (int *)mlp->step.p;
    a.lo = (const float *)mlp->lo.p;
    a.hi = (const float *)mlp->hi.p;
    a.X = X;
    a.y = y;
    a.batch = batch;
    a.lr = lr;
    a.loss = loss;
    a.grad_out = grad_out;
    k_mlp_step<<<1, 256, 0, ctx->stream>>>(a);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

int launch_mlp_infer(nb_ctx *ctx, const nb_mlp *mlp, const float *X, int batch, float *y) {
    MlpArgs a{};
    a.params = (float *)mlp->params.p;
    a.lo = (const float *)mlp->lo.p;
    a.hi = (const float *)mlp->hi.p;
    a.X = X;
    a.batch = batch;
    a.y_out = y;
    int nb = (batch + 3) / 4;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    k_mlp_infer<<<nb, 256, 0, ctx->stream>>>(a);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

}  // namespace mxn

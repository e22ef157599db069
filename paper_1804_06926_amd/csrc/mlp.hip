// The kernel-selector network: forward, backward and Adam kernels.
//
// A 6 -> 32 -> 32 -> 3 multilayer perceptron maps the features of a
// degree-pair bucket to one logit per intersection strategy; the pipeline
// takes the argmax per bucket. Weights are bfloat16 (rounded from a float32
// master copy), biases float32, accumulation float32. Training minimises the
// weighted softmax cross-entropy with Adam on the master copy; gradients pass
// through the bfloat16 rounding unchanged.
//
// The network is tiny (1379 parameters, at most 256 buckets per graph), so the
// kernels use one thread per sample or per parameter; gradient sums run over
// the batch in a fixed order, so a training step is deterministic.
#include <math.h>

#include "common.h"
#include "internal.h"
#include "mlp.h"

namespace tcx {

// float32 -> bfloat16 bits, round to nearest, ties to even; NaN kept quiet.
__device__ __forceinline__ uint16_t to_bf16(float x) {
    const uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x0040u);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct MlpShared {
    float W1[MLP_H * MLP_IN];
    float b1[MLP_H];
    float W2[MLP_H * MLP_H];
    float b2[MLP_H];
    float W3[MLP_OUT * MLP_H];
    float b3[MLP_OUT];
};

// Expand the compute copy (bf16 weights, f32 biases) into LDS as float.
__device__ void load_net(const MlpCompute* __restrict__ cw, MlpShared& S) {
    for (int i = threadIdx.x; i < MLP_H * MLP_IN; i += blockDim.x) S.W1[i] = from_bf16(cw->W1[i]);
    for (int i = threadIdx.x; i < MLP_H * MLP_H; i += blockDim.x) S.W2[i] = from_bf16(cw->W2[i]);
    for (int i = threadIdx.x; i < MLP_OUT * MLP_H; i += blockDim.x) S.W3[i] = from_bf16(cw->W3[i]);
    for (int i = threadIdx.x; i < MLP_H; i += blockDim.x) { S.b1[i] = cw->b1[i]; S.b2[i] = cw->b2[i]; }
    for (int i = threadIdx.x; i < MLP_OUT; i += blockDim.x) S.b3[i] = cw->b3[i];
    __syncthreads();
}

// One sample: dot products accumulate in input order, the bias is added last.
__device__ void net_forward(const MlpShared& S, const float* x, float* h1, float* h2, float* z) {
    for (int o = 0; o < MLP_H; ++o) {
        float acc = 0.f;
        for (int i = 0; i < MLP_IN; ++i) acc = fmaf(S.W1[o * MLP_IN + i], x[i], acc);
        acc += S.b1[o];
        h1[o] = acc > 0.f ? acc : 0.f;
    }
    for (int o = 0; o < MLP_H; ++o) {
        float acc = 0.f;
        for (int i = 0; i < MLP_H; ++i) acc = fmaf(S.W2[o * MLP_H + i], h1[i], acc);
        acc += S.b2[o];
        h2[o] = acc > 0.f ? acc : 0.f;
    }
    for (int o = 0; o < MLP_OUT; ++o) {
        float acc = 0.f;
        for (int i = 0; i < MLP_H; ++i) acc = fmaf(S.W3[o * MLP_H + i], h2[i], acc);
        z[o] = acc + S.b3[o];
    }
}

// Master (float32 parameter vector) -> compute copy.
__global__ __launch_bounds__(256) void k_mlp_cast(const float* __restrict__ master, MlpCompute* __restrict__ cw) {
    for (int p = threadIdx.x; p < MLP_NPARAM; p += 256) {
        const float x = master[p];
        if (p < MLP_OFF_B1) cw->W1[p - MLP_OFF_W1] = to_bf16(x);
        else if (p < MLP_OFF_W2) cw->b1[p - MLP_OFF_B1] = x;
        else if (p < MLP_OFF_B2) cw->W2[p - MLP_OFF_W2] = to_bf16(x);
        else if (p < MLP_OFF_W3) cw->b2[p - MLP_OFF_B2] = x;
        else if (p < MLP_OFF_B3) cw->W3[p - MLP_OFF_W3] = to_bf16(x);
        else cw->b3[p - MLP_OFF_B3] = x;
    }
}

__global__ __launch_bounds__(256) void k_mlp_forward(const MlpCompute* __restrict__ cw, const float* __restrict__ X,
                                                     int B, float* __restrict__ logits) {
    __shared__ MlpShared S;
    load_net(cw, S);
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= B) return;
    float x[MLP_IN], h1[MLP_H], h2[MLP_H], z[MLP_OUT];
    for (int i = 0; i < MLP_IN; ++i) x[i] = X[s * MLP_IN + i];
    net_forward(S, x, h1, h2, z);
    for (int o = 0; o < MLP_OUT; ++o) logits[s * MLP_OUT + o] = z[o];
}

// Per sample: forward, loss term, and the backpropagated errors of each layer.
__global__ __launch_bounds__(256) void k_mlp_fwdbwd(const MlpCompute* __restrict__ cw, const float* __restrict__ X,
                                                    const int32_t* __restrict__ y, const float* __restrict__ w, int B,
                                                    MlpActs acts) {
    __shared__ MlpShared S;
    load_net(cw, S);
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= B) return;
    float x[MLP_IN], h1[MLP_H], h2[MLP_H], z[MLP_OUT];
    for (int i = 0; i < MLP_IN; ++i) x[i] = X[s * MLP_IN + i];
    net_forward(S, x, h1, h2, z);
    const float ws = (w ? w[s] : 1.f) / (float)B;
    float zmax = z[0];
    for (int o = 1; o < MLP_OUT; ++o) zmax = fmaxf(zmax, z[o]);
    float e[MLP_OUT], se = 0.f;
    for (int o = 0; o < MLP_OUT; ++o) { e[o] = expf(z[o] - zmax); se += e[o]; }
    const int ys = min(max((int)y[s], 0), MLP_OUT - 1);   // labels are 0..2; clamp keeps indexing in range
    acts.loss[s] = ws * (logf(se) + zmax - z[ys]);
    float dz[MLP_OUT];
    for (int o = 0; o < MLP_OUT; ++o) dz[o] = ws * (e[o] / se - (o == ys ? 1.f : 0.f));
    float dh2[MLP_H], dh1[MLP_H];
    for (int j = 0; j < MLP_H; ++j) {
        float acc = 0.f;
        for (int o = 0; o < MLP_OUT; ++o) acc = fmaf(S.W3[o * MLP_H + j], dz[o], acc);
        dh2[j] = h2[j] > 0.f ? acc : 0.f;
    }
    for (int i = 0; i < MLP_H; ++i) {
        float acc = 0.f;
        for (int j = 0; j < MLP_H; ++j) acc = fmaf(S.W2[j * MLP_H + i], dh2[j], acc);
        dh1[i] = h1[i] > 0.f ? acc : 0.f;
    }
    for (int i = 0; i < MLP_H; ++i) {
        acts.h1[s * MLP_H + i] = h1[i];
        acts.h2[s * MLP_H + i] = h2[i];
        acts.dh1[s * MLP_H + i] = dh1[i];
        acts.dh2[s * MLP_H + i] = dh2[i];
    }
    for (int o = 0; o < MLP_OUT; ++o) acts.dz[s * MLP_OUT + o] = dz[o];
}

// One thread per parameter: gradient = sum over samples in order; thread
// MLP_NPARAM sums the loss terms.
__global__ __launch_bounds__(256) void k_mlp_param_grads(const float* __restrict__ X, int B, MlpActs acts,
                                                         float* __restrict__ grad, float* __restrict__ loss) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > MLP_NPARAM) return;
    float acc = 0.f;
    if (p == MLP_NPARAM) {
        for (int s = 0; s < B; ++s) acc += acts.loss[s];
        *loss = acc;
        return;
    }
    if (p < MLP_OFF_B1) {
        const int o = (p - MLP_OFF_W1) / MLP_IN, i = (p - MLP_OFF_W1) % MLP_IN;
        for (int s = 0; s < B; ++s) acc = fmaf(acts.dh1[s * MLP_H + o], X[s * MLP_IN + i], acc);
    } else if (p < MLP_OFF_W2) {
        const int o = p - MLP_OFF_B1;
        for (int s = 0; s < B; ++s) acc += acts.dh1[s * MLP_H + o];
    } else if (p < MLP_OFF_B2) {
        const int o = (p - MLP_OFF_W2) / MLP_H, i = (p - MLP_OFF_W2) % MLP_H;
        for (int s = 0; s < B; ++s) acc = fmaf(acts.dh2[s * MLP_H + o], acts.h1[s * MLP_H + i], acc);
    } else if (p < MLP_OFF_W3) {
        const int o = p - MLP_OFF_B2;
        for (int s = 0; s < B; ++s) acc += acts.dh2[s * MLP_H + o];
    } else if (p < MLP_OFF_B3) {
        const int o = (p - MLP_OFF_W3) / MLP_H, i = (p - MLP_OFF_W3) % MLP_H;
        for (int s = 0; s < B; ++s) acc = fmaf(acts.dz[s * MLP_OUT + o], acts.h2[s * MLP_H + i], acc);
    } else {
        const int o = p - MLP_OFF_B3;
        for (int s = 0; s < B; ++s) acc += acts.dz[s * MLP_OUT + o];
    }
    grad[p] = acc;
}

// Adam on the float32 master copy (bias-corrected moments).
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ master, const float* __restrict__ grad,
                                                  float* __restrict__ m, float* __restrict__ v, float lr, float beta1,
                                                  float beta2, float eps, float c1, float c2) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float g = grad[p];
    const float mp = beta1 * m[p] + (1.f - beta1) * g;
    const float vp = beta2 * v[p] + (1.f - beta2) * g * g;
    m[p] = mp;
    v[p] = vp;
    master[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// Bucket features (6 floats): the bucket's two degree classes and the log
// sizes of its work, from the statistics gathered by the pipeline: the
// LDS-bitmap windows its middle lists span (the bitmap strategy's set-up
// count, which grows with the rank range a list covers and so with the
// graph's size), in-edges, out-neighbours, and in-edges x out-degree.
__device__ void bucket_features(const Ctrl* ctrl, int b, float* f) {
    f[0] = (float)(b >> 4) / 14.f;
    f[1] = (float)(b & 15) / 15.f;
    f[2] = log2f(1.f + (float)ctrl->bucket_win[b]) / 32.f;
    f[3] = log2f(1.f + (float)ctrl->bucket_in[b]) / 32.f;
    f[4] = log2f(1.f + (float)ctrl->bucket_out[b]) / 32.f;
    f[5] = log2f(1.f + (float)ctrl->bucket_work[b]) / 48.f;
}

// SEL_G lanes per bucket: lane j of a group computes hidden units
// SEL_U * j .. SEL_U * j + SEL_U - 1 of each layer, and output j (j < 3), each
// as the same ordered dot product plus bias as net_forward, so the logits are
// bit-identical to it; the other lanes' units arrive by shuffles. Argmax ties
// go to the lower index.
constexpr int SEL_G = 8, SEL_U = MLP_H / SEL_G, SEL_NT = 256;
static_assert(MLP_H % SEL_G == 0 && MLP_OUT <= SEL_G && WAVE % SEL_G == 0, "selection lane layout");
__global__ __launch_bounds__(SEL_NT) void k_mlp_select(const MlpCompute* __restrict__ cw, Ctrl* ctrl,
                                                       uint8_t* __restrict__ choice) {
    __shared__ MlpShared S;
    load_net(cw, S);
    const int t = blockIdx.x * SEL_NT + threadIdx.x;
    const int b = t / SEL_G, j = t % SEL_G;   // NBUCKET * SEL_G threads in all
    const int lane0 = lane_id() - j;            // the group's first lane
    float x[MLP_IN];
    bucket_features(ctrl, b, x);
    if (j == 0)
        for (int i = 0; i < MLP_IN; ++i) ctrl->features[b][i] = x[i];
    float h1[SEL_U], h2[SEL_U];
#pragma unroll
    for (int u = 0; u < SEL_U; ++u) {
        const int o = SEL_U * j + u;
        float acc = 0.f;
        for (int i = 0; i < MLP_IN; ++i) acc = fmaf(S.W1[o * MLP_IN + i], x[i], acc);
        acc += S.b1[o];
        h1[u] = acc > 0.f ? acc : 0.f;
    }
    float hin[MLP_H];   // all of layer 1, in order
#pragma unroll
    for (int i = 0; i < MLP_H; ++i) hin[i] = __shfl(h1[i % SEL_U], lane0 + i / SEL_U, WAVE);
#pragma unroll
    for (int u = 0; u < SEL_U; ++u) {
        const int o = SEL_U * j + u;
        float acc = 0.f;
        for (int i = 0; i < MLP_H; ++i) acc = fmaf(S.W2[o * MLP_H + i], hin[i], acc);
        acc += S.b2[o];
        h2[u] = acc > 0.f ? acc : 0.f;
    }
#pragma unroll
    for (int i = 0; i < MLP_H; ++i) hin[i] = __shfl(h2[i % SEL_U], lane0 + i / SEL_U, WAVE);
    float z = 0.f;
    if (j < MLP_OUT) {
        for (int i = 0; i < MLP_H; ++i) z = fmaf(S.W3[j * MLP_H + i], hin[i], z);
        z += S.b3[j];
    }
    float zz[MLP_OUT];
#pragma unroll
    for (int o = 0; o < MLP_OUT; ++o) zz[o] = __shfl(z, lane0 + o, WAVE);
    if (j == 0) {
        int best = 0;
        for (int o = 1; o < MLP_OUT; ++o)
            if (zz[o] > zz[best]) best = o;
        choice[b] = (uint8_t)best;
    }
}

// Features only (heuristic and forced modes), for training data.
__global__ __launch_bounds__(NBUCKET) void k_bucket_features(Ctrl* ctrl) {
    float x[MLP_IN];
    bucket_features(ctrl, threadIdx.x, x);
    for (int i = 0; i < MLP_IN; ++i) ctrl->features[threadIdx.x][i] = x[i];
}

// ------------------------------------------------------------------ launchers
void mlp_cast(const float* master, MlpCompute* cw, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_cast, dim3(1), dim3(256), 0, s, master, cw);
}
void mlp_forward(const MlpCompute* cw, const float* X, int B, float* logits, hipStream_t s) {
    if (B > 0) hipLaunchKernelGGL(k_mlp_forward, dim3((B + 255) / 256), dim3(256), 0, s, cw, X, B, logits);
}
void mlp_gradient(const MlpCompute* cw, const float* X, const int32_t* y, const float* w, int B, const MlpActs& acts,
                  float* grad, float* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3((B + 255) / 256), dim3(256), 0, s, cw, X, y, w, B, acts);
    hipLaunchKernelGGL(k_mlp_param_grads, dim3((MLP_NPARAM + 1 + 255) / 256), dim3(256), 0, s, X, B, acts, grad,
                       loss);
}
void mlp_adam(float* master, const float* grad, float* m, float* v, float lr, int step, hipStream_t s) {
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, master, grad, m, v, lr, beta1,
                       beta2, eps, c1, c2);
}
void mlp_select(const MlpCompute* cw, Ctrl* ctrl, uint8_t* choice, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_select, dim3(NBUCKET * SEL_G / SEL_NT), dim3(SEL_NT), 0, s, cw, ctrl, choice);
}
void bucket_features_launch(Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(k_bucket_features, dim3(1), dim3(NBUCKET), 0, s, ctrl);
}

}  // namespace tcx

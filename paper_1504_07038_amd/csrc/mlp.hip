// Cost model of the schedule autotuner: a two-hidden-layer fp32 perceptron
// (ReLU units, one linear output) with its forward pass, its mean-squared-error
// gradient and an Adam update.  It predicts how long a decode schedule takes;
// it never touches pixel or bin bits.
//
//     z1 = W1 x + b1, h1 = max(z1, 0); z2 = W2 h1 + b2, h2 = max(z2, 0);
//     y = w3 . h2 + b3;  L = (1/N) sum_s (y_s - t_s)^2
//
// Gradients are the chain rule layer by layer (backpropagation, Rumelhart,
// Hinton and Williams 1986): with gy_s = 2 (y_s - t_s) / N,
//     dL/dw3 = sum gy h2, dL/dz2 = gy w3 [z2 > 0], dL/dW2 = sum dz2 h1^T,
//     dL/dz1 = W2^T dz2 [z1 > 0], dL/dW1 = sum dz1 x^T, biases the sums.
// Adam: Kingma and Ba, ICLR 2015, with bias correction.
//
// Sizes are tiny (D <= 16 inputs, H in {16, 32}), so these are plain FMA
// loops over parameters staged in LDS, not matrix-core tiles.  The gradient
// is summed without atomics: each workgroup accumulates its samples in a
// fixed order into its own partial vector, and a second kernel adds the
// partials in workgroup order, so results are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mj_internal.h"

namespace {

constexpr int kMaxIn = 16;
constexpr int kThreads = 256;
constexpr int kTileSamples = 32;       // samples staged per gradient tile
constexpr int kMaxPartials = 256;      // workgroups of the gradient pass

__host__ __device__ constexpr int np_of(int D, int H) { return H * D + H + H * H + H + H + 1; }

// Forward pass of one sample held in registers; params in LDS.
template <int H>
__device__ __forceinline__ float forward_one(const float *prm, int D, const float *x, float *h1,
                                             float *z2out) {
    const float *W1 = prm, *b1 = W1 + H * D, *W2 = b1 + H, *b2 = W2 + H * H, *w3 = b2 + H;
    const float b3 = w3[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        float z = b1[i];
#pragma unroll
        for (int j = 0; j < kMaxIn; ++j)
            if (j < D) z = fmaf(W1[i * D + j], x[j], z);
        h1[i] = z > 0.f ? z : 0.f;
    }
    float y = b3;
#pragma unroll 4
    for (int i = 0; i < H; ++i) {
        float z = b2[i];
#pragma unroll
        for (int j = 0; j < H; ++j) z = fmaf(W2[i * H + j], h1[j], z);
        z2out[i] = z;
        y = fmaf(w3[i], z > 0.f ? z : 0.f, y);
    }
    return y;
}

template <int H>
__global__ __launch_bounds__(kThreads) void mlp_forward_kernel(const float *params, int D,
                                                               const float *x, int64_t n,
                                                               float *y) {
    extern __shared__ float prm[];
    const int np = np_of(D, H);
    for (int i = threadIdx.x; i < np; i += blockDim.x) prm[i] = params[i];
    __syncthreads();
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        float xs[kMaxIn], h1[H], z2[H];
#pragma unroll
        for (int j = 0; j < kMaxIn; ++j) xs[j] = j < D ? x[s * D + j] : 0.f;
        y[s] = forward_one<H>(prm, D, xs, h1, z2);
    }
}

// Partial gradient of one workgroup's samples: tiles of kTileSamples samples;
// one thread per sample runs the forward and backward passes of its sample
// into LDS, then every thread adds the tile's terms of the parameters it owns
// (p = tid + kThreads * u), samples in order.  partial[g][np] holds the
// workgroup's share of N * L / N = sum of squared errors / N.
template <int H>
__global__ __launch_bounds__(kThreads) void mlp_grad_kernel(const float *params, int D,
                                                            const float *x, const float *t,
                                                            int64_t n, float *partial) {
    extern __shared__ float lds[];
    constexpr int PMAX = (np_of(kMaxIn, H) + kThreads - 1) / kThreads;   // params per thread
    const int np = np_of(D, H);
    float *prm = lds;                                   // np
    float *sx = prm + np;                               // kTileSamples x D
    float *sh1 = sx + kTileSamples * kMaxIn;            // kTileSamples x H
    float *sh2 = sh1 + kTileSamples * H;                // kTileSamples x H
    float *sg2 = sh2 + kTileSamples * H;                // dL/dz2
    float *sg1 = sg2 + kTileSamples * H;                // dL/dz1
    float *sgy = sg1 + kTileSamples * H;                // dL/dy
    for (int i = threadIdx.x; i < np; i += blockDim.x) prm[i] = params[i];
    const float *W2 = prm + H * D + H, *w3 = W2 + H * H + H;
    const float inv_n = 1.0f / (float)n;

    // what each owned parameter index is: segment and (i, j)
    float acc[PMAX];
    int seg[PMAX], pi[PMAX], pj[PMAX];
#pragma unroll
    for (int u = 0; u < PMAX; ++u) {
        acc[u] = 0.f;
        int p = threadIdx.x + kThreads * u;
        seg[u] = -1;
        pi[u] = pj[u] = 0;
        if (p >= np) continue;
        if (p < H * D) { seg[u] = 0; pi[u] = p / D; pj[u] = p % D; continue; }
        p -= H * D;
        if (p < H) { seg[u] = 1; pi[u] = p; continue; }
        p -= H;
        if (p < H * H) { seg[u] = 2; pi[u] = p / H; pj[u] = p % H; continue; }
        p -= H * H;
        if (p < H) { seg[u] = 3; pi[u] = p; continue; }
        p -= H;
        if (p < H) { seg[u] = 4; pi[u] = p; continue; }
        seg[u] = 5;
    }
    float sse = 0.f;
    __syncthreads();
    const int64_t tiles = (n + kTileSamples - 1) / kTileSamples;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t s0 = tile * kTileSamples;
        const int ns = (int)min((int64_t)kTileSamples, n - s0);
        if (threadIdx.x < ns) {
            const int k = threadIdx.x;
            const int64_t s = s0 + k;
            float xs[kMaxIn], h1[H], z2[H];
#pragma unroll
            for (int j = 0; j < kMaxIn; ++j) {
                xs[j] = j < D ? x[s * D + j] : 0.f;
                sx[k * kMaxIn + j] = xs[j];
            }
            const float y = forward_one<H>(prm, D, xs, h1, z2);
            const float e = y - t[s];
            sse = fmaf(e, e, sse);
            const float gy = 2.f * e * inv_n;
            sgy[k] = gy;
#pragma unroll
            for (int i = 0; i < H; ++i) {
                sh1[k * H + i] = h1[i];
                sh2[k * H + i] = z2[i] > 0.f ? z2[i] : 0.f;
                z2[i] = z2[i] > 0.f ? gy * w3[i] : 0.f;     // now dL/dz2
                sg2[k * H + i] = z2[i];
            }
#pragma unroll
            for (int j = 0; j < H; ++j) {
                float g = 0.f;
#pragma unroll
                for (int i = 0; i < H; ++i) g = fmaf(W2[i * H + j], z2[i], g);
                sg1[k * H + j] = h1[j] > 0.f ? g : 0.f;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PMAX; ++u) {
            const int i = pi[u], j = pj[u];
            float a = acc[u];
            switch (seg[u]) {
                case 0: for (int k = 0; k < ns; ++k) a = fmaf(sg1[k * H + i], sx[k * kMaxIn + j], a); break;
                case 1: for (int k = 0; k < ns; ++k) a += sg1[k * H + i]; break;
                case 2: for (int k = 0; k < ns; ++k) a = fmaf(sg2[k * H + i], sh1[k * H + j], a); break;
                case 3: for (int k = 0; k < ns; ++k) a += sg2[k * H + i]; break;
                case 4: for (int k = 0; k < ns; ++k) a = fmaf(sgy[k], sh2[k * H + i], a); break;
                case 5: for (int k = 0; k < ns; ++k) a += sgy[k]; break;
                default: break;
            }
            acc[u] = a;
        }
        __syncthreads();
    }
    float *out = partial + (int64_t)blockIdx.x * (np + 1);
#pragma unroll
    for (int u = 0; u < PMAX; ++u)
        if (seg[u] >= 0) out[threadIdx.x + kThreads * u] = acc[u];
    // squared errors: lanes 0..kTileSamples-1 hold them; add in lane order
    float *red = sx;
    red[threadIdx.x] = sse;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int k = 0; k < kTileSamples; ++k) s += red[k];
        out[np] = s * inv_n;
    }
}

__global__ void mlp_reduce_kernel(const float *partial, int groups, int width, float *grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= width) return;
    float s = 0.f;
    for (int g = 0; g < groups; ++g) s += partial[(int64_t)g * width + p];
    grad[p] = s;
}

__global__ void mlp_adam_kernel(float *params, const float *grad, float *m, float *v, int np,
                                float lr, float beta1, float beta2, float eps, float c1,
                                float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const float g = grad[p];
    const float mp = beta1 * m[p] + (1.f - beta1) * g;
    const float vp = beta2 * v[p] + (1.f - beta2) * g * g;
    m[p] = mp;
    v[p] = vp;
    params[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

bool shape_ok(int D, int H) { return D >= 1 && D <= kMaxIn && (H == 16 || H == 32); }

int groups_for(int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + kTileSamples - 1) / kTileSamples,
                                                        kMaxPartials));
}

size_t grad_lds(int D, int H) {
    return ((size_t)np_of(D, H) + kTileSamples * kMaxIn + 4 * kTileSamples * H + kTileSamples) *
           sizeof(float);
}

}  // namespace

extern "C" {

int32_t mojette_mlp_params(int32_t d_in, int32_t hidden) {
    return shape_ok(d_in, hidden) ? np_of(d_in, hidden) : -1;
}

int mojette_mlp_forward(const float *params, int32_t d_in, int32_t hidden, const float *x,
                        int64_t n, float *y, void *stream) {
    if (!shape_ok(d_in, hidden) || n < 0 || (n > 0 && (!params || !x || !y))) return MOJETTE_EINVAL;
    if (n == 0) return MOJETTE_OK;
    const int grid = (int)std::min<int64_t>((n + kThreads - 1) / kThreads, 1024);
    const size_t lds = (size_t)np_of(d_in, hidden) * sizeof(float);
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    switch (hidden) {
        case 16: hipLaunchKernelGGL(mlp_forward_kernel<16>, dim3(grid), dim3(kThreads), lds, s, params, d_in, x, n, y); break;
        default: hipLaunchKernelGGL(mlp_forward_kernel<32>, dim3(grid), dim3(kThreads), lds, s, params, d_in, x, n, y); break;
    }
    return mj::hip_status(hipGetLastError());
}

int64_t mojette_mlp_grad_workspace(int32_t d_in, int32_t hidden, int64_t n) {
    if (!shape_ok(d_in, hidden) || n < 1) return -1;
    return (int64_t)groups_for(n) * (np_of(d_in, hidden) + 1);
}

int mojette_mlp_grad(const float *params, int32_t d_in, int32_t hidden, const float *x,
                     const float *t, int64_t n, float *grad, float *workspace, void *stream) {
    if (!shape_ok(d_in, hidden) || n < 1 || !params || !x || !t || !grad || !workspace)
        return MOJETTE_EINVAL;
    const int groups = groups_for(n);
    const int width = np_of(d_in, hidden) + 1;
    const size_t lds = grad_lds(d_in, hidden);
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    switch (hidden) {
        case 16: hipLaunchKernelGGL(mlp_grad_kernel<16>, dim3(groups), dim3(kThreads), lds, s, params, d_in, x, t, n, workspace); break;
        default: hipLaunchKernelGGL(mlp_grad_kernel<32>, dim3(groups), dim3(kThreads), lds, s, params, d_in, x, t, n, workspace); break;
    }
    const int st = mj::hip_status(hipGetLastError());
    if (st != MOJETTE_OK) return st;
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((width + 255) / 256), dim3(256), 0, s, workspace,
                       groups, width, grad);
    return mj::hip_status(hipGetLastError());
}

int mojette_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t nparams,
                     float lr, float beta1, float beta2, float eps, int32_t step, void *stream) {
    if (!params || !grad || !m || !v || nparams < 1 || step < 1) return MOJETTE_EINVAL;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    (void)hipGetLastError();
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((nparams + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, params, grad, m, v, nparams, lr, beta1, beta2, eps,
                       c1, c2);
    return mj::hip_status(hipGetLastError());
}

}  // extern "C"

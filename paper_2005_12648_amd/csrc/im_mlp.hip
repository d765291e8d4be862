// im_mlp.hip -- the learned split's network: 1 -> 32 -> 1 ReLU, fp32.
//
// Not part of the paper.  The network maps a normalised diagonal x = k/N to a
// normalised co-rank y ~ i(k)/L_A; the split search (im_search.h) corrects
// its prediction to the exact co-rank.  Training labels come from the plain
// co-rank search on evenly spaced diagonals; the loss is the mean squared
// error; the optimiser is Adam.  Parameter layout: w1[H], b1[H], w2[H], b2.
#include "im_common.h"
#include "im_search.h"

namespace imerge {

constexpr int kMlpThreads = 256;
constexpr int kMlpOut = kMlpParams + 1;   // gradient entries + loss

// Partial gradients: block b accumulates samples b, b+G, ... and writes
// kMlpOut floats to partial[b * kMlpOut].
__global__ __launch_bounds__(kMlpThreads) void k_mlp_grad(const float *__restrict__ prm,
                                                          const float *__restrict__ xs,
                                                          const float *__restrict__ ts, int64_t m,
                                                          float *__restrict__ partial) {
    __shared__ float sp[kMlpParams];
    __shared__ float red[kMlpThreads / 64][kMlpOut];
    const int tid = threadIdx.x;
    for (int j = tid; j < kMlpParams; j += kMlpThreads) sp[j] = prm[j];
    __syncthreads();
    float g[kMlpOut];
#pragma unroll
    for (int j = 0; j < kMlpOut; ++j) g[j] = 0.0f;
    const float inv_m = 1.0f / (float)m;
    for (int64_t s = (int64_t)blockIdx.x * kMlpThreads + tid; s < m;
         s += (int64_t)gridDim.x * kMlpThreads) {
        const float x = xs[s];
        float y = sp[3 * kMlpHidden];
        float a[kMlpHidden];
#pragma unroll
        for (int h = 0; h < kMlpHidden; ++h) {
            float z = fmaf(sp[h], x, sp[kMlpHidden + h]);
            a[h] = fmaxf(z, 0.0f);
            y = fmaf(sp[2 * kMlpHidden + h], a[h], y);
        }
        const float r = y - ts[s];
        const float dy = 2.0f * r * inv_m;
#pragma unroll
        for (int h = 0; h < kMlpHidden; ++h) {
            const float dz = a[h] > 0.0f ? dy * sp[2 * kMlpHidden + h] : 0.0f;
            g[h] = fmaf(dz, x, g[h]);                       // d/d w1
            g[kMlpHidden + h] += dz;                         // d/d b1
            g[2 * kMlpHidden + h] = fmaf(dy, a[h], g[2 * kMlpHidden + h]);   // d/d w2
        }
        g[3 * kMlpHidden] += dy;                             // d/d b2
        g[kMlpParams] = fmaf(r * r, inv_m, g[kMlpParams]);   // loss
    }
    // wave reduction, then across the block's waves
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int j = 0; j < kMlpOut; ++j) {
        float v = g[j];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave][j] = v;
    }
    __syncthreads();
    for (int j = tid; j < kMlpOut; j += kMlpThreads) {
        float v = 0.0f;
        for (int q = 0; q < kMlpThreads / 64; ++q) v += red[q][j];
        partial[(int64_t)blockIdx.x * kMlpOut + j] = v;
    }
}

// Fixed-order sum of the block partials (deterministic).
__global__ void k_mlp_reduce(const float *__restrict__ partial, int nb, float *__restrict__ grad,
                             float *__restrict__ loss) {
    for (int j = threadIdx.x; j < kMlpOut; j += blockDim.x) {
        float v = 0.0f;
        for (int b = 0; b < nb; ++b) v += partial[(int64_t)b * kMlpOut + j];
        if (j < kMlpParams) grad[j] = v;
        else if (loss) *loss = v;
    }
}

// Adam (Kingma & Ba): bias-corrected first/second moment estimates.
__global__ void k_mlp_adam(float *__restrict__ prm, const float *__restrict__ g,
                           float *__restrict__ mo, float *__restrict__ ve, float lr, int step) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)step);
    const float c2 = 1.0f - powf(b2, (float)step);
    for (int j = threadIdx.x; j < kMlpParams; j += blockDim.x) {
        float gj = g[j];
        float m = b1 * mo[j] + (1.0f - b1) * gj;
        float v = b2 * ve[j] + (1.0f - b2) * gj * gj;
        mo[j] = m;
        ve[j] = v;
        prm[j] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
    }
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ prm, const float *__restrict__ xs, int64_t m,
                              float *__restrict__ ys) {
    __shared__ MlpDev sm;
    for (int j = threadIdx.x; j < kMlpParams; j += blockDim.x) sm.p[j] = prm[j];
    __syncthreads();
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < m;
         s += (int64_t)gridDim.x * blockDim.x)
        ys[s] = mlp_eval(&sm, xs[s]);
}

// Training diagonals: k_p = floor((p + 1/2) * N / m), x_p = k_p / N.
__global__ void k_mlp_samples(int64_t n, int64_t m, int64_t *__restrict__ ks, float *__restrict__ xs) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m;
         p += (int64_t)gridDim.x * blockDim.x) {
        int64_t k = (int64_t)(((double)p + 0.5) * (double)n / (double)m);
        if (k > n) k = n;
        ks[p] = k;
        xs[p] = (float)((double)k / (double)n);
    }
}

__global__ void k_mlp_targets(const int64_t *__restrict__ is, int64_t m, int64_t la,
                              float *__restrict__ ts) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m;
         p += (int64_t)gridDim.x * blockDim.x)
        ts[p] = la > 0 ? (float)((double)is[p] / (double)la) : 0.0f;
}

// Prediction errors in A elements over the training diagonals: their mean
// (err_scale, a statistic) and, per bucket of x, the bracket half-width that
// the searches start from: 1.25 x the largest error seen in the bucket or
// its two neighbours, plus 32 elements (fp32 resolution of x and y at
// 2^29 elements).  A bucket with no sample takes the largest error overall.
// The brackets are estimates between samples; the searches check both ends.
__global__ __launch_bounds__(1024) void k_mlp_errscale(const float *__restrict__ prm, const int64_t *__restrict__ ks,
                               const int64_t *__restrict__ is, int64_t m, int64_t la, int64_t lb,
                               MlpDev *__restrict__ model) {
    __shared__ MlpDev sm;
    __shared__ double red[1024];
    __shared__ int bmax[kErrBuckets];     // float bits of non-negative errors (-1: none)
    for (int j = threadIdx.x; j < kMlpParams; j += blockDim.x) sm.p[j] = prm[j];
    for (int j = threadIdx.x; j < kErrBuckets; j += blockDim.x) bmax[j] = -1;
    __syncthreads();
    const int64_t n = la + lb;
    double acc = 0.0;
    for (int64_t p = threadIdx.x; p < m; p += blockDim.x) {
        const float x = n > 0 ? (float)((double)ks[p] / (double)n) : 0.0f;
        const double pred = (double)mlp_eval(&sm, x) * (double)la;
        double err = fabs(pred - (double)is[p]);
        if (!(err == err) || err > 1e30) err = 1e30;
        acc += err;
        int b = (int)(x * (float)kErrBuckets);
        b = b < 0 ? 0 : (b >= kErrBuckets ? kErrBuckets - 1 : b);
        atomicMax(&bmax[b], __float_as_int((float)err));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    // largest error over all buckets (for buckets without samples)
    __shared__ int gmax;
    if (threadIdx.x == 0) gmax = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < kErrBuckets; j += blockDim.x)
        if (bmax[j] >= 0) atomicMax(&gmax, bmax[j]);
    __syncthreads();
    for (int j = threadIdx.x; j < kMlpParams; j += blockDim.x) model->p[j] = prm[j];
    for (int j = threadIdx.x; j < kErrBuckets; j += blockDim.x) {
        int v = -1;
        for (int q = j - 1; q <= j + 1; ++q)
            if (q >= 0 && q < kErrBuckets && bmax[q] > v) v = bmax[q];
        const float worst = __int_as_float(v >= 0 ? v : gmax);
        const float hw = 1.25f * worst + 32.0f;
        model->err_b[j] = hw < kErrUnknown ? hw : kErrUnknown;
    }
    if (threadIdx.x == 0) {
        double mean = m > 0 ? red[0] / (double)m : 1.0;
        if (!(mean >= 1.0)) mean = 1.0;
        if (mean > 1e15) mean = 1e15;
        model->err_scale = (float)mean;
    }
}

int mlp_grad_blocks(int64_t m) {
    int64_t b = (m + kMlpThreads * 8 - 1) / (kMlpThreads * 8);
    if (b < 1) b = 1;
    if (b > 256) b = 256;
    return (int)b;
}

hipError_t launch_mlp_grad(const float *d_params, const float *d_x, const float *d_t, int64_t m,
                           float *d_partial, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblocks), dim3(kMlpThreads), 0, s, d_params, d_x, d_t, m,
                       d_partial);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(const float *d_partial, int nblocks, float *d_grad, float *d_loss,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_reduce, dim3(1), dim3(128), 0, s, d_partial, nblocks, d_grad, d_loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, float lr,
                           int step, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_adam, dim3(1), dim3(128), 0, s, d_params, d_grad, d_m, d_v, lr, step);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *d_params, const float *d_x, int64_t m, float *d_y,
                              hipStream_t s) {
    int64_t g = (m + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_mlp_forward, dim3((int)g), dim3(256), 0, s, d_params, d_x, m, d_y);
    return hipGetLastError();
}

hipError_t launch_mlp_samples(int key, const void *, int64_t la, int64_t lb, int64_t m,
                              int64_t *d_k, float *d_x, hipStream_t s) {
    (void)key;
    int64_t g = (m + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_mlp_samples, dim3((int)g), dim3(256), 0, s, la + lb, m, d_k, d_x);
    return hipGetLastError();
}

hipError_t launch_mlp_targets(const int64_t *d_i, int64_t m, int64_t la, float *d_t, hipStream_t s) {
    int64_t g = (m + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_mlp_targets, dim3((int)g), dim3(256), 0, s, d_i, m, la, d_t);
    return hipGetLastError();
}

hipError_t launch_mlp_errscale(const float *d_params, const int64_t *d_k, const int64_t *d_i,
                               int64_t m, int64_t la, int64_t lb, MlpDev *d_model, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_errscale, dim3(1), dim3(1024), 0, s, d_params, d_k, d_i, m, la, lb,
                       d_model);
    return hipGetLastError();
}

}  // namespace imerge

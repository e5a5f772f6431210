// Leaf-plane encoding (FP32 -> storage type, padded rows), decoding, the
// photometric loss of a training batch, the optimiser updates of the leaf
// parameters (Adam, RMSProp) and the density signal.
#include <hip/hip_runtime.h>

#include "dot_device.h"

namespace dot {

// dst[r][0..cols) = round(src[r][0..cols)), padding columns zeroed.
template <int DT>
__global__ void encode_kernel(const float* __restrict__ src, void* __restrict__ dst, int64_t rows, int cols,
                              int stride) {
    int64_t n = rows * stride;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i / stride;
        int c = (int)(i - r * stride);
        float v = c < cols ? src[r * cols + c] : 0.f;
        if constexpr (DT == DOT_F32)
            static_cast<float*>(dst)[i] = v;
        else if constexpr (DT == DOT_F16)
            static_cast<uint16_t*>(dst)[i] = f32_to_f16(v);
        else
            static_cast<uint16_t*>(dst)[i] = f32_to_bf16(v);
    }
}

template <int DT>
__global__ void decode_kernel(const void* __restrict__ src, float* __restrict__ dst, int64_t rows, int cols,
                              int stride) {
    int64_t n = rows * cols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i / cols;
        int c = (int)(i - r * cols);
        int64_t j = r * stride + c;
        float v;
        if constexpr (DT == DOT_F32)
            v = static_cast<const float*>(src)[j];
        else if constexpr (DT == DOT_F16)
            v = f16_to_f32(static_cast<const uint16_t*>(src)[j]);
        else
            v = bf16_to_f32(static_cast<const uint16_t*>(src)[j]);
        dst[i] = v;
    }
}

static unsigned grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t launch_encode_planes(int storage, const float* src, void* dst, int64_t rows, int cols, int stride,
                                hipStream_t s) {
    if (rows == 0) return hipSuccess;
    dim3 g(grid_for(rows * stride));
    if (storage == DOT_F32)
        hipLaunchKernelGGL(encode_kernel<DOT_F32>, g, dim3(256), 0, s, src, dst, rows, cols, stride);
    else if (storage == DOT_F16)
        hipLaunchKernelGGL(encode_kernel<DOT_F16>, g, dim3(256), 0, s, src, dst, rows, cols, stride);
    else
        hipLaunchKernelGGL(encode_kernel<DOT_BF16>, g, dim3(256), 0, s, src, dst, rows, cols, stride);
    return hipGetLastError();
}

hipError_t launch_decode_planes(int storage, const void* src, float* dst, int64_t rows, int cols, int stride,
                                hipStream_t s) {
    if (rows == 0) return hipSuccess;
    dim3 g(grid_for(rows * cols));
    if (storage == DOT_F32)
        hipLaunchKernelGGL(decode_kernel<DOT_F32>, g, dim3(256), 0, s, src, dst, rows, cols, stride);
    else if (storage == DOT_F16)
        hipLaunchKernelGGL(decode_kernel<DOT_F16>, g, dim3(256), 0, s, src, dst, rows, cols, stride);
    else
        hipLaunchKernelGGL(decode_kernel<DOT_BF16>, g, dim3(256), 0, s, src, dst, rows, cols, stride);
    return hipGetLastError();
}

// Adam (adam_update) on every parameter.  Parameter j < L is sigma[j]; j >= L is SH coefficient (j-L) of the dense
// [L][3K] layout, stored at row stride `stride` in the plane.
__global__ void adam_kernel(float* __restrict__ sigma, float* __restrict__ sh, const float* __restrict__ gs,
                            const float* __restrict__ gh, float* __restrict__ ms, float* __restrict__ vs,
                            float* __restrict__ mh, float* __restrict__ vh, int64_t L, int nv, int stride,
                            dot_adam_params p, float bc1, float bc2) {
    int64_t n = L * (1 + nv);
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        float g, m, v, lr;
        float* theta;
        float *mp, *vp;
        if (j < L) {
            g = gs[j];
            mp = &ms[j];
            vp = &vs[j];
            theta = &sigma[j];
            lr = p.lr_sigma;
        } else {
            int64_t q = j - L;
            int64_t r = q / nv;
            int c = (int)(q - r * nv);
            g = gh[q];
            mp = &mh[q];
            vp = &vh[q];
            theta = &sh[r * stride + c];
            lr = p.lr_sh;
        }
        m = *mp;
        v = *vp;
        float th = *theta;
        adam_update(th, m, v, g, lr, p.beta1, p.beta2, p.eps, bc1, bc2);
        *mp = m;
        *vp = v;
        *theta = th;
    }
}

hipError_t launch_adam(const dot_tree& t, const float* gs, const float* gh, float* ms, float* vs, float* mh,
                       float* vh, const dot_adam_params& p, hipStream_t s) {
    int nv = 3 * (t.degree + 1) * (t.degree + 1);
    int64_t n = t.n_leaves * (1 + nv);
    float bc1, bc2;
    adam_bias_corrections(p, bc1, bc2);
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, s, static_cast<float*>(t.sigma),
                       static_cast<float*>(t.sh), gs, gh, ms, vs, mh, vh, t.n_leaves, nv, t.sh_stride, p, bc1,
                       bc2);
    return hipGetLastError();
}

// RMSProp: v = alpha v + (1-alpha) g^2; theta -= lr * g / (sqrt(v) + eps).
__global__ void rmsprop_kernel(float* __restrict__ sigma, float* __restrict__ sh, const float* __restrict__ gs,
                               const float* __restrict__ gh, float* __restrict__ vs, float* __restrict__ vh, int64_t L,
                               int nv, int stride, dot_rmsprop_params p) {
    int64_t n = L * (1 + nv);
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        float g, lr;
        float *theta, *vp;
        if (j < L) {
            g = gs[j];
            vp = &vs[j];
            theta = &sigma[j];
            lr = p.lr_sigma;
        } else {
            int64_t q = j - L;
            int64_t r = q / nv;
            int c = (int)(q - r * nv);
            g = gh[q];
            vp = &vh[q];
            theta = &sh[r * stride + c];
            lr = p.lr_sh;
        }
        float v = *vp, th = *theta;
        rmsprop_update(th, v, g, lr, p.alpha, p.eps);
        *vp = v;
        *theta = th;
    }
}

hipError_t launch_rmsprop(const dot_tree& t, const float* gs, const float* gh, float* vs, float* vh,
                          const dot_rmsprop_params& p, hipStream_t s) {
    int nv = 3 * (t.degree + 1) * (t.degree + 1);
    int64_t n = t.n_leaves * (1 + nv);
    hipLaunchKernelGGL(rmsprop_kernel, dim3(grid_for(n)), dim3(256), 0, s, static_cast<float*>(t.sigma),
                       static_cast<float*>(t.sh), gs, gh, vs, vh, t.n_leaves, nv, t.sh_stride, p);
    return hipGetLastError();
}

template <int DT>
__global__ void sigma_signal_kernel(const void* __restrict__ sig, int64_t L, float* __restrict__ out) {
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < L; l += (int64_t)gridDim.x * blockDim.x)
        out[l] = fmaxf(load_sigma<DT>(sig, l), 0.f);
}

hipError_t launch_sigma_signal(const dot_tree& t, float* out, hipStream_t s) {
    dim3 g(grid_for(t.n_leaves));
    if (t.storage == DOT_F32)
        hipLaunchKernelGGL(sigma_signal_kernel<DOT_F32>, g, dim3(256), 0, s, t.sigma, t.n_leaves, out);
    else if (t.storage == DOT_F16 || t.storage == DOT_PAL16)
        hipLaunchKernelGGL(sigma_signal_kernel<DOT_F16>, g, dim3(256), 0, s, t.sigma, t.n_leaves, out);
    else
        hipLaunchKernelGGL(sigma_signal_kernel<DOT_BF16>, g, dim3(256), 0, s, t.sigma, t.n_leaves, out);
    return hipGetLastError();
}

// Squared error of a ray batch and its gradient.  One block partial per
// workgroup, combined with a double atomic into *loss (zeroed by the first
// kernel of the same stream).
__global__ void zero_f64_kernel(double* p) { *p = 0.0; }

// Each workgroup ends with one FP64 atomic on the single loss value, and those
// atomics queue on one address, so the grid is kept to at most MSE_BLOCKS
// large workgroups (a 2^20-ray batch: 256 atomics instead of 4096).
constexpr int MSE_THREADS = 1024;
constexpr int MSE_BLOCKS = 256;

__global__ __launch_bounds__(MSE_THREADS) void mse_kernel(const float* __restrict__ pred, const float* __restrict__ target,
                                                  const int64_t* __restrict__ idx, int64_t n, double gscale,
                                                  const double* __restrict__ gmul, float* __restrict__ grad,
                                                  double* __restrict__ loss, double lscale) {
    __shared__ double part[MSE_THREADS / WAVE];
    double acc = 0.0;
    if (gmul) gscale *= *gmul;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = idx ? idx[r] : r;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double e = (double)pred[3 * r + c] - (double)target[3 * t + c];   // exact
            if (grad) grad[3 * r + c] = (float)(gscale * e);
            acc += e * e;
        }
    }
    if (!loss) return;
    for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_down(acc, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int w = 0; w < MSE_THREADS / WAVE; ++w) b += part[w];
        atomicAdd(loss, b * lscale);
    }
}

hipError_t launch_mse(const float* pred, const float* target, const int64_t* idx, int64_t n, const double* gmul,
                      float* grad, double* loss, hipStream_t s) {
    if (loss) {
        hipLaunchKernelGGL(zero_f64_kernel, dim3(1), dim3(1), 0, s, loss);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n == 0) return hipSuccess;
    int64_t g = (n + MSE_THREADS - 1) / MSE_THREADS;
    if (g > MSE_BLOCKS) g = MSE_BLOCKS;
    const double gscale = 2.0 / (3.0 * (double)n);
    hipLaunchKernelGGL(mse_kernel, dim3((unsigned)g), dim3(MSE_THREADS), 0, s, pred, target, idx, n, gscale, gmul,
                       grad, loss, 1.0 / (3.0 * (double)n));
    return hipGetLastError();
}

}  // namespace dot

// Small device utilities: strided 2-D copies (layout changes between the
// column-major QR panels and the row-major TT cores) and a deterministic
// two-level sum of squares (the residual estimate ||S||_F of Sec. 3.3 and
// the norm estimate of Remark 1).
#include "kernels.hpp"

namespace ttr {
namespace {

__global__ void __launch_bounds__(256) copy2d_kernel(const double* __restrict__ src, int64_t ssr,
                                                     int64_t ssc, double* __restrict__ dst,
                                                     int64_t dsr, int64_t dsc, int rows, int cols,
                                                     double scale) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * cols) return;
    // Walk the destination's contiguous dimension with consecutive threads.
    int r, c;
    if (dsc == 1) {
        r = (int)(t / cols);
        c = (int)(t - (int64_t)r * cols);
    } else {
        c = (int)(t / rows);
        r = (int)(t - (int64_t)c * rows);
    }
    dst[(size_t)r * dsr + (size_t)c * dsc] = scale * src[(size_t)r * ssr + (size_t)c * ssc];
}

__global__ void __launch_bounds__(256) axpby2d_kernel(const double* __restrict__ src, int64_t ssr, int64_t ssc,
                                                      double* __restrict__ dst, int64_t dsr, int64_t dsc, int rows,
                                                      int cols, double alpha, double beta) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * cols) return;
    int r, c;
    if (dsc == 1) {
        r = (int)(t / cols);
        c = (int)(t - (int64_t)r * cols);
    } else {
        c = (int)(t / rows);
        r = (int)(t - (int64_t)c * rows);
    }
    double* d = dst + (size_t)r * dsr + (size_t)c * dsc;
    double v = src ? alpha * src[(size_t)r * ssr + (size_t)c * ssc] : 0.0;
    if (beta != 0.0) v += beta * (*d);
    *d = v;
}

constexpr int kSumBlocks = 1024;

__global__ void __launch_bounds__(256) sumsq_kernel(const double* __restrict__ a, int64_t sr,
                                                    int64_t sc, int rows, int cols,
                                                    double* __restrict__ out,
                                                    double* __restrict__ partial, int* counter) {
    __shared__ double red[4];
    __shared__ int last;
    const int64_t total = (int64_t)rows * cols;
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if ((sr == 1 && sc == rows) || (sc == 1 && sr == cols)) {
        // contiguous (the estimator's residual block): no index arithmetic
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
            const double v = a[t];
            s += v * v;
        }
    } else {
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
            int r, c;
            if (sr == 1) {
                c = (int)(t / rows);
                r = (int)(t - (int64_t)c * rows);
            } else {
                r = (int)(t / cols);
                c = (int)(t - (int64_t)r * cols);
            }
            const double v = a[(size_t)r * sr + (size_t)c * sc];
            s += v * v;
        }
    }
    s = block_sum256(s, red);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = s;
        __threadfence();
        last = (atomicAdd(counter, 1) == (int)gridDim.x - 1);
    }
    __syncthreads();
    if (last) {
        __threadfence();
        double v = 0.0;
        for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x)
            v += __builtin_nontemporal_load(&partial[i]);
        v = block_sum256(v, red);
        if (threadIdx.x == 0) {
            *out = v;
            *counter = 0;
        }
    }
}

}  // namespace

void launch_copy2d(const double* src, int64_t ssr, int64_t ssc, double* dst, int64_t dsr,
                   int64_t dsc, int rows, int cols, double scale, hipStream_t s) {
    const int64_t work = (int64_t)rows * cols;
    if (work <= 0) return;
    hipLaunchKernelGGL(copy2d_kernel, dim3(ceil_div(work, 256)), dim3(256), 0, s, src, ssr, ssc,
                       dst, dsr, dsc, rows, cols, scale);
    TTR_CHECK_LAUNCH();
}

void launch_axpby2d(const double* src, int64_t ssr, int64_t ssc, double* dst, int64_t dsr, int64_t dsc, int rows,
                    int cols, double alpha, double beta, hipStream_t s) {
    const int64_t work = (int64_t)rows * cols;
    if (work <= 0) return;
    hipLaunchKernelGGL(axpby2d_kernel, dim3(ceil_div(work, 256)), dim3(256), 0, s, src, ssr, ssc, dst, dsr, dsc,
                       rows, cols, alpha, beta);
    TTR_CHECK_LAUNCH();
}

void launch_sumsq(const double* a, int64_t sr, int64_t sc, int rows, int cols, double* out,
                  double* partial, int* counter, hipStream_t s) {
    const int64_t total = (int64_t)rows * cols;
    int blocks = (int)std::min<int64_t>(kSumBlocks, std::max<int64_t>(1, (total + 1023) / 1024));
    hipLaunchKernelGGL(sumsq_kernel, dim3(blocks), dim3(256), 0, s, a, sr, sc, rows, cols, out,
                       partial, counter);
    TTR_CHECK_LAUNCH();
}

}  // namespace ttr

// Image-wide error statistics in FP64 (reporting only): per-block partial
// sums of img, img^2, (img - ref)^2, relative squared error and its count,
// and the max absolute error; the host adds the partials.
#include "rlc_internal.h"

namespace rlc {

namespace {

constexpr int kBlock = 256;
constexpr int kFields = 6;

__global__ void __launch_bounds__(kBlock) k_image_error(const float* __restrict__ img, const float* __restrict__ ref,
                                                        uint32_t n, double* __restrict__ partial) {
    __shared__ double s[kFields][kBlock];
    double acc[kFields] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        double a = (double)img[i], r = (double)ref[i];
        double e = a - r;
        acc[0] += a;
        acc[1] += a * a;
        acc[2] += e * e;
        if (r != 0.0) {
            acc[3] += (e * e) / (r * r);
            acc[4] += 1.0;
        }
        double ae = e < 0.0 ? -e : e;
        acc[5] = ae > acc[5] ? ae : acc[5];
    }
    for (int f = 0; f < kFields; ++f) s[f][threadIdx.x] = acc[f];
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            for (int f = 0; f < 5; ++f) s[f][threadIdx.x] += s[f][threadIdx.x + off];
            double m = s[5][threadIdx.x + off];
            if (m > s[5][threadIdx.x]) s[5][threadIdx.x] = m;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int f = 0; f < kFields; ++f) partial[kFields * blockIdx.x + f] = s[f][0];
}

}  // namespace

hipError_t launch_image_error(const float* img, const float* ref, uint32_t n, double* partial, uint32_t nblocks,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_image_error, dim3(nblocks), dim3(kBlock), 0, s, img, ref, n, partial);
    return hipGetLastError();
}

}  // namespace rlc

// General box bounds l_j <= x_j <= u_j (paper, Section 2: the substitution
// x := x - l moves every lower bound to 0, with d := d - A l and r := u - l).
// Two small kernels around the bounded path: the substitution itself, and
// adding l back to each verified row.
#include "msp_internal.h"

namespace msp {

namespace {
constexpr long long kBoxLimit = 1ll << 24;  // |l_j|, |u_j|: keeps d - A l and the embedding exact in int64

// d' = d - A l and r = u - l; status[0] = 1 when some bound is outside
// what the bounded path accepts (u_j - l_j in 1..255, |l_j|, |u_j| <= 2^24).
__global__ void box_setup_kernel(int m, int n, const int32_t *A, const int64_t *d, const int32_t *lo,
                                 const int32_t *hi, int64_t *d_out, int32_t *r_out, int *status) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const long long l = lo[j], u = hi[j];
        const long long r = u - l;
        if (r < 1 || r > 255 || l > kBoxLimit || l < -kBoxLimit || u > kBoxLimit || u < -kBoxLimit)
            atomicOr(&bad, 1);
        r_out[j] = (int32_t)r;
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        long long acc = d[i];
        for (int j = 0; j < n; ++j) acc -= (long long)A[(size_t)i * n + j] * (long long)lo[j];
        d_out[i] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) status[0] = bad;
}

// x_j = x'_j + l_j for `rows` rows of n variables.
__global__ void box_shift_kernel(int64_t rows, int n, const uint8_t *xs, const int32_t *lo, int32_t *x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < rows * n) x[i] = (int32_t)xs[i] + lo[i % n];
}
}  // namespace

hipError_t launch_box_setup(int m, int n, const int32_t *A, const int64_t *d, const int32_t *lo, const int32_t *hi,
                            int64_t *d_out, int32_t *r_out, int *status, hipStream_t st) {
    hipLaunchKernelGGL(box_setup_kernel, dim3(1), dim3(256), 0, st, m, n, A, d, lo, hi, d_out, r_out, status);
    return hipGetLastError();
}

hipError_t launch_box_shift(int64_t rows, int n, const uint8_t *xs, const int32_t *lo, int32_t *x, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    const int64_t tot = rows * n;
    hipLaunchKernelGGL(box_shift_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, rows, n, xs, lo, x);
    return hipGetLastError();
}

}  // namespace msp

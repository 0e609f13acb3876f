// Gram-Schmidt orthogonalisation of a kernel lattice basis (paper, eq. (4);
// step 3 of Algorithm 1), FP64.
//
// One 64-lane wave per basis.  Lane l holds columns l and l+64 of the vector
// being orthogonalised (dim <= 128).  Modified Gram-Schmidt: b_i is reduced
// against b_hat_0, b_hat_1, ... in turn; in exact arithmetic the coefficient
// <v, b_hat_j> / ||b_hat_j||^2 of the partly reduced v equals
// mu_ij = <b_i, b_hat_j> / ||b_hat_j||^2 because the b_hat are orthogonal.
// The finished rows stay in LDS (k x dim doubles <= 128 KiB) and are written
// out at the end.
#include "msp_internal.h"

namespace msp {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(64) gram_schmidt_kernel(GsArgs a) {
    extern __shared__ __align__(16) double s_bh[];   // k x dim
    const int k = a.k, dim = a.dim;
    const int l0 = threadIdx.x, l1 = threadIdx.x + 64;
    double *s_beta = s_bh + (size_t)k * dim;
    for (int i = 0; i < k; ++i) {
        double v0 = l0 < dim ? (double)a.basis[(size_t)i * dim + l0] : 0.0;
        double v1 = l1 < dim ? (double)a.basis[(size_t)i * dim + l1] : 0.0;
        for (int j = 0; j < i; ++j) {
            const double b0 = l0 < dim ? s_bh[(size_t)j * dim + l0] : 0.0;
            const double b1 = l1 < dim ? s_bh[(size_t)j * dim + l1] : 0.0;
            const double dot = wave_sum(v0 * b0 + v1 * b1);
            const double m = dot / s_beta[j];
            if (threadIdx.x == 0) a.mu[(size_t)i * k + j] = m;
            v0 -= m * b0;
            v1 -= m * b1;
        }
        const double bi = wave_sum(v0 * v0 + v1 * v1);
        if (l0 < dim) s_bh[(size_t)i * dim + l0] = v0;
        if (l1 < dim) s_bh[(size_t)i * dim + l1] = v1;
        if (threadIdx.x == 0) {
            s_beta[i] = bi;
            a.beta[i] = bi;
            a.mu[(size_t)i * k + i] = 1.0;
            if (!(bi > 0.0)) *a.err = 1;
        }
        for (int j = i + 1 + threadIdx.x; j < k; j += 64) a.mu[(size_t)i * k + j] = 0.0;
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < k * dim; idx += 64) a.bhat[idx] = s_bh[idx];
}

hipError_t launch_gram_schmidt(const GsArgs &a, hipStream_t st) {
    if (a.k < 1 || a.dim < 1 || a.dim > 128 || a.k > 128) return hipErrorInvalidValue;
    size_t lds = ((size_t)a.k * a.dim + a.k) * sizeof(double);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)gram_schmidt_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gram_schmidt_kernel, dim3(1), dim3(64), lds, st, a);
    return hipGetLastError();
}

}  // namespace msp

// Shuffled copies of an instance for the first-solution restarts (paper,
// Section 4: the method run on randomly reordered input bases).  Copy r
// permutes the variables: its column j is column perm[r][j] of A, so its
// solution x' maps back to x[perm[r][j]] = x'[j].
#include "msp_internal.h"

namespace msp {

// out[r] (m x n) = A[:, perm[r]] for r < copies
__global__ void permute_cols_kernel(const int32_t *A, int m, int n, const int32_t *perm, int copies, int32_t *out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)m * n;
    if (e >= per * copies) return;
    const int r = (int)(e / per);
    const int64_t ij = e - (int64_t)r * per;
    const int i = (int)(ij / n), j = (int)(ij - (int64_t)i * n);
    out[e] = A[(int64_t)i * n + perm[(int64_t)r * n + j]];
}

// x[s][perm[j]] = xc[s][j] for s < rows
__global__ void unpermute_rows_kernel(const uint8_t *xc, int64_t rows, int n, const int32_t *perm, uint8_t *x) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * n) return;
    const int64_t s = e / n;
    const int j = (int)(e - s * n);
    x[s * n + perm[j]] = xc[e];
}

hipError_t launch_permute_cols(const int32_t *A, int m, int n, const int32_t *perm, int copies, int32_t *out,
                               hipStream_t st) {
    const int64_t total = (int64_t)m * n * copies;
    if (total <= 0) return hipSuccess;
    const int B = 256;
    hipLaunchKernelGGL(permute_cols_kernel, dim3((unsigned)((total + B - 1) / B)), dim3(B), 0, st, A, m, n, perm,
                       copies, out);
    return hipGetLastError();
}

hipError_t launch_unpermute_rows(const uint8_t *xc, int64_t rows, int n, const int32_t *perm, uint8_t *x,
                                 hipStream_t st) {
    const int64_t total = rows * n;
    if (total <= 0) return hipSuccess;
    const int B = 256;
    hipLaunchKernelGGL(unpermute_rows_kernel, dim3((unsigned)((total + B - 1) / B)), dim3(B), 0, st, xc, rows, n, perm,
                       x);
    return hipGetLastError();
}

}  // namespace msp

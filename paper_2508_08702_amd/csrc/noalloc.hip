// msp_reduce_noalloc: steps 1-2 of Algorithm 1 (the eq. (2) embedding, LLL,
// kernel extraction) without any device allocation, for callers that cannot
// allocate (code under stream capture, tight serving loops).
//
// The reduction's scratch -- one launch descriptor (status, kernel vectors
// found, iterations) and the (n+1) x (m+n+1) int64 embedding workspace -- lives
// in the file-scope device array `scratch` below, sized for the largest
// accepted instance (n <= MSP_MAX_N, m <= n).  Each GPU holds its own copy of
// the array until the process ends; its address is looked up once per device
// (hipGetSymbolAddress with that device current) and only that address is
// handed to kernels.  Every call on one GPU shares the array and finds the
// previous call's contents in it; the descriptor is rewritten by a kernel at
// the start of each call, and the LLL kernel builds the embedding in the
// workspace from scratch.  Calls that overlap on one GPU (different host
// threads, or streams running concurrently) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/msp.h"
#include "msp_internal.h"

namespace msp {
namespace {
constexpr size_t kDescBytes = 256;  // LllDesc, padded to the workspace's alignment
constexpr size_t kWorkBytes = (size_t)(MSP_MAX_N + 1) * (2 * MSP_MAX_N + 1) * sizeof(long long);
constexpr size_t kScratchBytes = kDescBytes + kWorkBytes;  // 261,376 bytes
static_assert(sizeof(LllDesc) <= kDescBytes, "descriptor does not fit its slot");
}  // namespace
}  // namespace msp

static __device__ __align__(256) unsigned char scratch[msp::kScratchBytes];

namespace msp {
namespace {
constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices];
int g_scratch_rc[kMaxDevices];
std::once_flag g_scratch_once[kMaxDevices];

__global__ void noalloc_desc_kernel(LllDesc *d, int m, int n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        d->m = m;
        d->n = n;
        d->A_off = 0;
        d->d_off = 0;
        d->work_off = 0;
        d->out_off = 0;
        d->status = 0;
        d->kout = 0;
        d->iters = 0;
    }
}

int noalloc_status(int32_t st) {
    switch (st) {
        case 0: return MSP_OK;
        case -2: return MSP_E_RANK;
        case -3: return MSP_E_NOT_ISOLATED;
        case -4: return MSP_E_OVERFLOW;
        default: return MSP_E_NUMERIC;
    }
}
}  // namespace
}  // namespace msp

extern "C" int msp_reduce_noalloc(int m, int n, const int32_t *A_dev, const int64_t *d_dev, const msp_params *pin,
                                  int64_t *basis_dev, int *k_out, void *stream) {
    using namespace msp;
    if (!A_dev || !d_dev || !basis_dev || !k_out) return MSP_E_ARG;
    if (m < 1 || n < 1 || m > n || n > MSP_MAX_N) return MSP_E_ARG;
    msp_params p;
    msp_params_default(&p);
    if (pin) p = *pin;
    if (p.N < 1 || !(p.delta > 0.25 && p.delta < 1.0)) return MSP_E_ARG;
    if (p.bkz_block != 0) return MSP_E_ARG;  // BKZ needs more scratch than this entry point holds
    const size_t need = kDescBytes + (size_t)(n + 1) * (size_t)(m + n + 1) * sizeof(long long);
    if (need > kScratchBytes) return MSP_E_ARG;
    *k_out = 0;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MSP_E_DEVICE;
    // the array's address on this device, looked up once with the device current
    std::call_once(g_scratch_once[dev], [dev]() {
        g_scratch_rc[dev] = (int)hipGetSymbolAddress(&g_scratch[dev], HIP_SYMBOL(scratch));
    });
    if (g_scratch_rc[dev] != (int)hipSuccess || !g_scratch[dev]) return MSP_E_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    LllDesc *dd = reinterpret_cast<LllDesc *>(g_scratch[dev]);
    long long *work = reinterpret_cast<long long *>(reinterpret_cast<unsigned char *>(g_scratch[dev]) + kDescBytes);
    hipLaunchKernelGGL(noalloc_desc_kernel, dim3(1), dim3(64), 0, st, dd, m, n);
    if (hipGetLastError() != hipSuccess) return MSP_E_DEVICE;
    LllArgs la{};
    la.m = &dd->m;
    la.n = &dd->n;
    la.A = A_dev;
    la.A_off = &dd->A_off;
    la.d = d_dev;
    la.d_off = &dd->d_off;
    la.N = p.N;
    la.delta = p.delta;
    la.max_iters = 2000000;
    la.work = work;
    la.work_off = &dd->work_off;
    la.out = basis_dev;
    la.out_off = &dd->out_off;
    la.status = &dd->status;
    la.kout = &dd->kout;
    la.iters = &dd->iters;
    la.stride = (int)(sizeof(LllDesc) / sizeof(int32_t));
    la.cvec = nullptr;
    la.rmax = 1;
    if (launch_lll(la, 1, n, st) != hipSuccess) return MSP_E_DEVICE;
    LllDesc h{};
    if (hipMemcpyAsync(&h, dd, sizeof(LllDesc), hipMemcpyDeviceToHost, st) != hipSuccess) return MSP_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return MSP_E_DEVICE;
    const int s = noalloc_status(h.status);
    if (s != MSP_OK) return s;
    *k_out = h.kout;
    return MSP_OK;
}

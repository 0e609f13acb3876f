// Orders of the subtree roots for first-solution search.
//
// The paper's enumeration visits subtree roots depth first (Section 2; the
// roots come from tree partitioning, Section 4).  For mode "first" the roots
// may be taken in any order without changing the result set, so two other
// orders are offered:
//   * discrepancy order: fewest departures from the first (closest-to-centre)
//     zig-zag value above the root first -- limited discrepancy search
//     (Section 3) applied to the order of the roots;
//   * learned order: a small MLP (16 -> 64 -> 64 -> 1, ReLU, BF16 weights,
//     FP32 accumulation) scores every root from features of its prefix and
//     the roots are taken best score first.
// This file holds the per-root feature and label kernels, the MLP forward,
// gradient and Adam kernels, and the sorts that turn scores into an order.
#include <rocprim/device/device_radix_sort.hpp>

#include "enum_rules.h"
#include "msp_internal.h"

namespace msp {

namespace {

__device__ __forceinline__ float bf16_rne(float x) {
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7f800000u) == 0x7f800000u) return x;  // inf / nan unchanged
    b += 0x7fffu + ((b >> 16) & 1u);
    return __uint_as_float(b & 0xffff0000u);
}

}  // namespace

// ---------------------------------------------------------------------------
// Root features.  For root r at level L with prefix u_{k-1..L}:
//   per level j (top first): centre y_j (the enumeration's fixed order),
//   x_j = u_j + y_j,
//   zig-zag rank of u_j (its position in the sequence u1, u1+s, u1-s, ...,
//   or u_j itself while every higher u is zero).
//   f0  l / R                      f8  min(max |u_j|, 4) / 4
//   f1  l / ||w||_1 (0 if w = 0)   f9  x_L^2 beta_L / R
//   f2  min(||w||_inf, 4) / 4      f10 min(|x_L|, 2) / 2
//   f3  mean rank                  f11 (L/k) ln(max((R-l)/R, 1e-6)) / 8
//   f4  fraction of levels with rank > 0 (discrepancies)
//   f5  min(max rank, 8) / 8       f12 r / np (depth-first position)
//   f6  fraction of u_j != 0       f13 fraction of coordinates with |w_j| > 17/16
//   f7  mean |u_j|                 f14 L / k        f15 m / 16
// Computed in FP64, stored as FP32 (np x 16, row-major).
__global__ void root_feat_kernel(FeatArgs a) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.np) return;
    const int k = a.k, L = a.L;
    const int8_t *u = a.roots.u + r * k;
    const double *w = a.roots.w + r;  // column-major: element j at w[j * wcap]
    const int64_t wcap = a.roots.wcap;
    const double l = a.roots.l[r];
    const double R = a.R;
    double rank_sum = 0.0;
    int disc = 0, rmax = 0, nz = 0, usum = 0, umax = 0;
    bool tz = true;
    double xL = 0.0, eL = 0.0;
    for (int j = k - 1; j >= L; --j) {
        const double y = centre_natural(u, a.mu, k, j);
        const int uj = u[j];
        int rank;
        if (tz) {
            rank = uj;
        } else {
            const Zig z = zig_init(y, false);
            const int o = uj - z.u1;
            const int ao = o < 0 ? -o : o;
            rank = o == 0 ? 0 : (((o > 0) == (z.s > 0)) ? 2 * ao - 1 : 2 * ao);
        }
        rank_sum += (double)rank;
        disc += rank > 0;
        rmax = rank > rmax ? rank : rmax;
        const int au = uj < 0 ? -uj : uj;
        nz += uj != 0;
        usum += au;
        umax = au > umax ? au : umax;
        if (j == L) {
            xL = add_rn((double)uj, y);
            eL = mul_rn(mul_rn(xL, xL), a.beta[j]);
        }
        tz = tz && uj == 0;
    }
    double l1 = 0.0, linf = 0.0;
    int big = 0;
    for (int j = 0; j < a.dim; ++j) {
        const double v = fabs(w[(size_t)j * wcap]);
        l1 += v;
        linf = v > linf ? v : linf;
        big += v > 1.0625;  // clear of +-1, a value projected coordinates often take exactly
    }
    const double lv = (double)(k - L);
    double f[16];
    f[0] = l / R;
    f[1] = l1 > 0.0 ? l / l1 : 0.0;
    f[2] = fmin(linf, 4.0) / 4.0;
    f[3] = rank_sum / lv;
    f[4] = (double)disc / lv;
    f[5] = (double)(rmax < 8 ? rmax : 8) / 8.0;
    f[6] = (double)nz / lv;
    f[7] = (double)usum / lv;
    f[8] = (double)(umax < 4 ? umax : 4) / 4.0;
    f[9] = eL / R;
    f[10] = fmin(fabs(xL), 2.0) / 2.0;
    f[11] = ((double)L / (double)k) * log(fmax((R - l) / R, 1e-6)) / 8.0;
    f[12] = (double)r / (double)a.np;
    f[13] = (double)big / (double)a.dim;
    f[14] = (double)L / (double)k;
    f[15] = (double)a.m / 16.0;
    float *o = a.feat + r * kNumFeat;
#pragma unroll
    for (int q = 0; q < kNumFeat; ++q) o[q] = (float)f[q];
}

hipError_t launch_root_features(const FeatArgs &a, hipStream_t st) {
    if (a.np <= 0) return hipSuccess;
    const int B = 256;
    hipLaunchKernelGGL(root_feat_kernel, dim3((unsigned)((a.np + B - 1) / B)), dim3(B), 0, st, a);
    return hipGetLastError();
}

// label[r] = 1 iff some recorded solution has root r's prefix (levels >= L):
// a solution lies in that subtree.
__global__ void root_label_kernel(Frontier roots, int64_t np, int k, int L, const int8_t *sol_u, int64_t nsol,
                                  uint8_t *label) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= np) return;
    const int8_t *u = roots.u + r * k;
    uint8_t hit = 0;
    for (int64_t s = 0; s < nsol && !hit; ++s) {
        const int8_t *v = sol_u + s * k;
        bool eq = true;
        for (int j = L; j < k && eq; ++j) eq = v[j] == u[j];
        hit = eq;
    }
    label[r] = hit;
}

hipError_t launch_root_labels(Frontier roots, int64_t np, int k, int L, const int8_t *sol_u, int64_t nsol,
                              uint8_t *label, hipStream_t st) {
    if (np <= 0) return hipSuccess;
    const int B = 256;
    hipLaunchKernelGGL(root_label_kernel, dim3((unsigned)((np + B - 1) / B)), dim3(B), 0, st, roots, np, k, L, sol_u,
                       nsol, label);
    return hipGetLastError();
}

// Discrepancy order key: minus the prefix's discrepancies, the rank sum
// recovered from the mean rank (an exact small integer in FP32), so a
// descending stable sort takes the fewest first and keeps depth-first order
// among equals.
__global__ void disc_key_kernel(const float *feat, int64_t np, int levels, float *key) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= np) return;
    key[r] = -rintf(feat[r * kNumFeat + 3] * (float)levels);
}

hipError_t launch_disc_keys(const float *feat, int64_t np, int levels, float *key, hipStream_t st) {
    if (np <= 0) return hipSuccess;
    const int B = 256;
    hipLaunchKernelGGL(disc_key_kernel, dim3((unsigned)((np + B - 1) / B)), dim3(B), 0, st, feat, np, levels, key);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MLP.  Parameter vector (FP32 master copy, BF16-rounded copy `wq` used by
// every kernel): W1[64][16] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3.
//   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = W3 . h2 + b3.
// Sums run over the input index in ascending order, accumulated in FP32.
namespace {
constexpr int kH = kHidden;
constexpr int OW1 = 0, OB1 = kH * kNumFeat, OW2 = OB1 + kH, OB2 = OW2 + kH * kH, OW3 = OB2 + kH, OB3 = OW3 + kH;
static_assert(OB3 + 1 == kNumParams, "parameter layout");

__device__ __forceinline__ void load_weights(float *s_w, const float *wq) {
    for (int i = threadIdx.x; i < kNumParams; i += blockDim.x) s_w[i] = wq[i];
    __syncthreads();
}

__device__ __forceinline__ float layer1(const float *s_w, const float *x, int o) {
    float acc = s_w[OB1 + o];
#pragma unroll
    for (int i = 0; i < kNumFeat; ++i) acc = fmaf(s_w[OW1 + o * kNumFeat + i], x[i], acc);
    return acc > 0.0f ? acc : 0.0f;
}

__device__ __forceinline__ float layer2(const float *s_w, const float *h1, int o) {
    float acc = s_w[OB2 + o];
    const float4 *row = reinterpret_cast<const float4 *>(s_w + OW2 + o * kH);
#pragma unroll
    for (int i = 0; i < kH / 4; ++i) {
        const float4 q = row[i];
        acc = fmaf(q.x, h1[4 * i], acc);
        acc = fmaf(q.y, h1[4 * i + 1], acc);
        acc = fmaf(q.z, h1[4 * i + 2], acc);
        acc = fmaf(q.w, h1[4 * i + 3], acc);
    }
    return acc > 0.0f ? acc : 0.0f;
}
}  // namespace

__global__ void __launch_bounds__(256) mlp_score_kernel(const float *wq, const float *feat, int64_t count,
                                                        float *logit) {
    __shared__ __align__(16) float s_w[kNumParams + 3];
    load_weights(s_w, wq);
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    float x[kNumFeat], h1[kH];
#pragma unroll
    for (int i = 0; i < kNumFeat; ++i) x[i] = feat[r * kNumFeat + i];
#pragma unroll
    for (int o = 0; o < kH; ++o) h1[o] = layer1(s_w, x, o);
    float z = s_w[OB3];
    for (int o = 0; o < kH; ++o) z = fmaf(s_w[OW3 + o], layer2(s_w, h1, o), z);
    logit[r] = z;
}

hipError_t launch_mlp_score(const float *wq, const float *feat, int64_t count, float *logit, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int B = 256;
    hipLaunchKernelGGL(mlp_score_kernel, dim3((unsigned)((count + B - 1) / B)), dim3(B), 0, st, wq, feat, count,
                       logit);
    return hipGetLastError();
}

// Gradient of the weighted logistic loss over one mini-batch:
//   loss = (1/B) sum_s c_s (softplus(z_s) - y_s z_s),  c_s = pos_weight if
//   y_s = 1 else 1, B = samples in the batch.
// One wave handles 64 samples: phase 1 runs each sample's forward and
// backward pass and keeps its activations and deltas in LDS (rows of 65
// floats: conflict-free both ways); phase 2 sums every parameter's gradient
// over the 64 samples (fixed order) and writes one partial row per wave.
// Batch b of an epoch covers perm[b*batch .. ) (identity when perm is null);
// b = (*step) mod steps_per_epoch, or 0 without a step counter.
namespace {
constexpr int kGS = 64;       // samples per wave
constexpr int kRow = kH + 1;  // LDS row stride (floats)
}  // namespace

__global__ void __launch_bounds__(kGS) mlp_grad_kernel(MlpGradArgs a) {
    __shared__ __align__(16) float s_w[kNumParams + 3];
    __shared__ float s_x[kGS * (kNumFeat + 1)];
    __shared__ float s_h1[kGS * kRow], s_h2[kGS * kRow], s_d2[kGS * kRow], s_d1[kGS * kRow];
    __shared__ float s_dz[kGS], s_loss[kGS];
    load_weights(s_w, a.wq);
    const int s = threadIdx.x;
    int64_t start = 0;
    if (a.step) start = (int64_t)((*a.step) % (unsigned long long)a.steps_per_epoch) * a.batch;
    const int64_t bend = start + a.batch < a.count ? start + a.batch : a.count;
    const float inv_b = 1.0f / (float)(bend - start);
    const int64_t pos = start + (int64_t)blockIdx.x * kGS + s;
    const bool act = pos < bend;
    float x[kNumFeat], h1[kH];
    float dz = 0.0f, lossv = 0.0f;
    if (act) {
        const int64_t g = a.perm ? (int64_t)a.perm[pos] : pos;
#pragma unroll
        for (int i = 0; i < kNumFeat; ++i) x[i] = a.feat[g * kNumFeat + i];
#pragma unroll
        for (int o = 0; o < kH; ++o) h1[o] = layer1(s_w, x, o);
        float z = s_w[OB3];
        for (int o = 0; o < kH; ++o) {
            const float h2 = layer2(s_w, h1, o);
            s_h2[s * kRow + o] = h2;
            z = fmaf(s_w[OW3 + o], h2, z);
        }
        const float y = a.label[g] ? 1.0f : 0.0f;
        const float c = a.label[g] ? a.pos_weight : 1.0f;
        const float sig = 1.0f / (1.0f + expf(-z));
        const float sp = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
        dz = c * (sig - y) * inv_b;
        lossv = c * (sp - y * z) * inv_b;
    } else {
#pragma unroll
        for (int i = 0; i < kNumFeat; ++i) x[i] = 0.0f;
#pragma unroll
        for (int o = 0; o < kH; ++o) h1[o] = 0.0f;
        for (int o = 0; o < kH; ++o) s_h2[s * kRow + o] = 0.0f;
    }
#pragma unroll
    for (int i = 0; i < kNumFeat; ++i) s_x[s * (kNumFeat + 1) + i] = x[i];
#pragma unroll
    for (int o = 0; o < kH; ++o) s_h1[s * kRow + o] = h1[o];
    s_dz[s] = dz;
    s_loss[s] = lossv;
    // dh2 = dz W3 (h2 > 0); dh1 = (W2^T dh2) (h1 > 0)
    float d1[kH];
#pragma unroll
    for (int i = 0; i < kH; ++i) d1[i] = 0.0f;
    for (int o = 0; o < kH; ++o) {
        const float h2 = s_h2[s * kRow + o];
        const float d2 = h2 > 0.0f ? dz * s_w[OW3 + o] : 0.0f;
        s_d2[s * kRow + o] = d2;
        const float4 *row = reinterpret_cast<const float4 *>(s_w + OW2 + o * kH);
#pragma unroll
        for (int i = 0; i < kH / 4; ++i) {
            const float4 q = row[i];
            d1[4 * i] = fmaf(q.x, d2, d1[4 * i]);
            d1[4 * i + 1] = fmaf(q.y, d2, d1[4 * i + 1]);
            d1[4 * i + 2] = fmaf(q.z, d2, d1[4 * i + 2]);
            d1[4 * i + 3] = fmaf(q.w, d2, d1[4 * i + 3]);
        }
    }
#pragma unroll
    for (int i = 0; i < kH; ++i) s_d1[s * kRow + i] = h1[i] > 0.0f ? d1[i] : 0.0f;
    __syncthreads();
    // phase 2: per-parameter sums over the 64 samples
    float *out = a.partial + (size_t)blockIdx.x * kPartialStride;
    for (int p = s; p <= kNumParams; p += kGS) {
        float acc = 0.0f;
        if (p < OB1) {
            const int o = p / kNumFeat, i = p % kNumFeat;
            for (int q = 0; q < kGS; ++q) acc = fmaf(s_d1[q * kRow + o], s_x[q * (kNumFeat + 1) + i], acc);
        } else if (p < OW2) {
            const int o = p - OB1;
            for (int q = 0; q < kGS; ++q) acc += s_d1[q * kRow + o];
        } else if (p < OB2) {
            const int o = (p - OW2) / kH, i = (p - OW2) % kH;
            for (int q = 0; q < kGS; ++q) acc = fmaf(s_d2[q * kRow + o], s_h1[q * kRow + i], acc);
        } else if (p < OW3) {
            const int o = p - OB2;
            for (int q = 0; q < kGS; ++q) acc += s_d2[q * kRow + o];
        } else if (p < OB3) {
            const int o = p - OW3;
            for (int q = 0; q < kGS; ++q) acc = fmaf(s_dz[q], s_h2[q * kRow + o], acc);
        } else if (p == OB3) {
            for (int q = 0; q < kGS; ++q) acc += s_dz[q];
        } else {  // p == kNumParams: the loss
            for (int q = 0; q < kGS; ++q) acc += s_loss[q];
        }
        out[p] = acc;
    }
}

hipError_t launch_mlp_grad(const MlpGradArgs &a, int waves, hipStream_t st) {
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)waves), dim3(kGS), 0, st, a);
    return hipGetLastError();
}

// Sum the per-wave partial rows (fixed order): grad[p] for p < kNumParams,
// the loss into *loss.
__global__ void grad_sum_kernel(const float *partial, int waves, float *grad, float *loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNumParams) return;
    float acc = 0.0f;
    for (int b = 0; b < waves; ++b) acc += partial[(size_t)b * kPartialStride + p];
    if (p < kNumParams)
        grad[p] = acc;
    else
        *loss = acc;
}

hipError_t launch_grad_sum(const float *partial, int waves, float *grad, float *loss, hipStream_t st) {
    hipLaunchKernelGGL(grad_sum_kernel, dim3((kNumParams + 256) / 256), dim3(256), 0, st, partial, waves, grad, loss);
    return hipGetLastError();
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the summed
// partial gradients; step t = *step + 1.  Writes the FP32 master weights and
// their BF16 rounding.  The loss of the batch is added to
// loss_acc[(t-1) / steps_per_epoch] / steps_per_epoch.
__global__ void adam_kernel(AdamArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNumParams) return;
    float g = 0.0f;
    for (int b = 0; b < a.waves; ++b) g += a.partial[(size_t)b * kPartialStride + p];
    const unsigned long long t0 = *a.step;
    if (p == kNumParams) {
        a.loss_acc[t0 / (unsigned long long)a.steps_per_epoch] += g / (float)a.steps_per_epoch;
        return;
    }
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float t = (float)(t0 + 1);
    const float mm = b1 * a.m[p] + (1.0f - b1) * g;
    const float vv = b2 * a.v[p] + (1.0f - b2) * g * g;
    a.m[p] = mm;
    a.v[p] = vv;
    const float mh = mm / (1.0f - powf(b1, t));
    const float vh = vv / (1.0f - powf(b2, t));
    const float w = a.master[p] - a.lr * mh / (sqrtf(vh) + eps);
    a.master[p] = w;
    a.wq[p] = bf16_rne(w);
}

__global__ void step_inc_kernel(unsigned long long *step) {
    if (threadIdx.x == 0) *step += 1ull;
}

hipError_t launch_adam(const AdamArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(adam_kernel, dim3((kNumParams + 256) / 256), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(step_inc_kernel, dim3(1), dim3(64), 0, st, a.step);
    return hipGetLastError();
}

__global__ void bf16_round_kernel(const float *master, float *wq) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNumParams) wq[p] = bf16_rne(master[p]);
}

hipError_t launch_bf16_round(const float *master, float *wq, hipStream_t st) {
    hipLaunchKernelGGL(bf16_round_kernel, dim3((kNumParams + 255) / 256), dim3(256), 0, st, master, wq);
    return hipGetLastError();
}

// Epoch shuffle: key_i = splitmix64(seed, epoch, i) (upper 32 bits), index i.
__global__ void shuffle_keys_kernel(uint32_t *keys, int32_t *idx, int64_t count, unsigned long long seed,
                                    int epoch) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    unsigned long long z = seed + 0x9e3779b97f4a7c15ull * ((unsigned long long)epoch * 0x100000001ull + i + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    keys[i] = (uint32_t)(z >> 32);
    idx[i] = (int32_t)i;
}

__global__ void count_pos_kernel(const uint8_t *label, int64_t count, unsigned long long *npos) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool p = i < count && label[i] != 0;
    const unsigned long long m = __ballot(p);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(npos, (unsigned long long)__popcll(m));
}

hipError_t launch_count_pos(const uint8_t *label, int64_t count, unsigned long long *npos, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(count_pos_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, label, count, npos);
    return hipGetLastError();
}

__global__ void iota64_kernel(int64_t *v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = i;
}

// Stable descending sort of scores -> root order (indices).  Temporary
// storage: *temp of *temp_bytes, grown by the caller when the query says so.
hipError_t sort_scores_desc(void *temp, size_t *temp_bytes, const float *key_in, float *key_out, int64_t *idx_in,
                            int64_t *idx_out, int64_t n, hipStream_t st) {
    if (temp == nullptr)
        return rocprim::radix_sort_pairs_desc(nullptr, *temp_bytes, key_in, key_out, idx_in, idx_out, (size_t)n, 0,
                                              32, st);
    hipLaunchKernelGGL(iota64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, idx_in, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return rocprim::radix_sort_pairs_desc(temp, *temp_bytes, key_in, key_out, idx_in, idx_out, (size_t)n, 0, 32,
                                          st);
}

// Ascending sort of indices (restores depth-first order of a selection).
hipError_t sort_idx_asc(void *temp, size_t *temp_bytes, const int64_t *in, int64_t *out, int64_t n, hipStream_t st) {
    return rocprim::radix_sort_keys(temp, *temp_bytes, in, out, (size_t)n, 0, 64, st);
}

hipError_t shuffle_perm(void *temp, size_t *temp_bytes, uint32_t *keys, uint32_t *keys_out, int32_t *idx,
                        int32_t *perm, int64_t n, unsigned long long seed, int epoch, hipStream_t st) {
    if (temp == nullptr)
        return rocprim::radix_sort_pairs(nullptr, *temp_bytes, keys, keys_out, idx, perm, (size_t)n, 0, 32, st);
    hipLaunchKernelGGL(shuffle_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, keys, idx, n, seed,
                       epoch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return rocprim::radix_sort_pairs(temp, *temp_bytes, keys, keys_out, idx, perm, (size_t)n, 0, 32, st);
}

}  // namespace msp

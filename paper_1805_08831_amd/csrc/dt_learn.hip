// Learned insertion scheduler (not in the paper): per-point features, a small MLP
// 16 -> 64 -> 64 -> 3 with BF16 weights and FP32 accumulation, its training kernels, and
// the logs of plain runs it is trained on.  The MLP only orders insertions and picks walk
// starts; every geometric decision is still taken by the exact predicates, so the
// triangulation does not depend on it.
//
// Outputs: y[0] = predicted log2(1 + attempts) of the point (its conflict / cavity cost);
// y[1], y[2] = logits of the walk-start bucket (0: nearest inserted curve neighbour,
// 1: the anchor of the previous level).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dt_internal.h"

namespace dtk {

// ------------------------------------------------------------------ bf16

// round-to-nearest-even fp32 -> bf16 (inputs are finite)
__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------------ features

// log2 of the distance from p to record q in grid cells of the cloud (scale s), or -8 when q
// is not a record of the same cloud of this call
__device__ __forceinline__ float ldist(const Vert &a, const Vert *__restrict__ V, uint32_t q, bool ok, double s) {
    if (!ok) return -8.0f;
    const Vert b = V[q];
    const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    const double d2 = (dx * dx + dy * dy + dz * dz) * s * s;
    return d2 > 0.0 ? (float)(0.5 * log2(d2)) : -8.0f;
}

// Features of the records [base, base + n): distances to the curve neighbours at +-1, 2, 4,
// 8, 16 and to the anchor (log2, grid cells), BRIO level and its share of the cloud,
// position in the cloud's box.
__global__ void k_features(const Vert *__restrict__ V, uint64_t base, uint64_t n, const Cloud *__restrict__ clouds,
                           const uint32_t *__restrict__ anchor, const uint8_t *__restrict__ level, int L,
                           float *__restrict__ feat) {
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = (uint32_t)(base + i);
    const Vert a = V[p];
    const Cloud cl = clouds[a.idx >> 32];
    const double s = cl.box[3];
    float f[NFEAT];
    int k = 0;
    for (int d = 1; d <= 16; d <<= 1) {
        f[k++] = ldist(a, V, p + d, p + d < cl.hi, s);
        f[k++] = ldist(a, V, p - d, p >= cl.lo + d, s);
    }
    const uint32_t q = anchor[i];
    f[k++] = ldist(a, V, q, q != NONE, s);
    f[k++] = L > 1 ? (float)level[i] / (float)(L - 1) : 0.0f;
    const double nc = (double)(cl.hi - cl.lo);
    f[k++] = (float)log2(fmin(2048.0 * pow(7.0, (double)level[i]), nc) / nc);
    const double cells = ldexp(1.0, (int)cl.m);
    f[k++] = (float)((a.x - cl.box[0]) * s / cells);
    f[k++] = (float)((a.y - cl.box[1]) * s / cells);
    f[k++] = (float)((a.z - cl.box[2]) * s / cells);
    for (int j = 0; j < NFEAT; ++j) feat[i * NFEAT + j] = f[j];
}

hipError_t launch_features(const Vert *V, uint64_t base, uint64_t n, const Cloud *clouds, const uint32_t *anchor,
                           const uint8_t *level, int L, float *feat, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_features<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(V, base, n, clouds, anchor, level, L, feat);
    return hipGetLastError();
}

// ------------------------------------------------------------------ MLP

// parameter offsets in the fp32 / bf16 weight vectors
constexpr int OW1 = 0, OB1 = OW1 + NFEAT * NHID, OW2 = OB1 + NHID, OB2 = OW2 + NHID * NHID, OW3 = OB2 + NHID,
              OB3 = OW3 + NHID * NOUT;
static_assert(OB3 + NOUT == NPARAM, "parameter layout");

__device__ __forceinline__ float relu(float x) { return x > 0.0f ? x : 0.0f; }

// forward pass of one sample with bf16 weights w (in LDS), fp32 accumulation
__device__ __forceinline__ void mlp_forward(const uint16_t *w, const float *x, float *h1, float *h2, float *y) {
    for (int j = 0; j < NHID; ++j) {
        float acc = bf2f(w[OB1 + j]);
        for (int k = 0; k < NFEAT; ++k) acc += x[k] * bf2f(w[OW1 + k * NHID + j]);
        h1[j] = relu(acc);
    }
    for (int j = 0; j < NHID; ++j) {
        float acc = bf2f(w[OB2 + j]);
        for (int k = 0; k < NHID; ++k) acc += h1[k] * bf2f(w[OW2 + k * NHID + j]);
        h2[j] = relu(acc);
    }
    for (int j = 0; j < NOUT; ++j) {
        float acc = bf2f(w[OB3 + j]);
        for (int k = 0; k < NHID; ++k) acc += h2[k] * bf2f(w[OW3 + k * NOUT + j]);
        y[j] = acc;
    }
}

// y[i] = MLP(feat[i]), one thread per sample; the bf16 weights are staged in LDS
__global__ __launch_bounds__(256) void k_mlp_infer(const uint16_t *__restrict__ wbf, const float *__restrict__ feat,
                                                   uint64_t n, float *__restrict__ y) {
    __shared__ uint16_t w[NPARAM];
    for (int k = threadIdx.x; k < NPARAM; k += blockDim.x) w[k] = wbf[k];
    __syncthreads();
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[NFEAT], h1[NHID], h2[NHID], o[NOUT];
    for (int k = 0; k < NFEAT; ++k) x[k] = feat[i * NFEAT + k];
    mlp_forward(w, x, h1, h2, o);
    for (int k = 0; k < NOUT; ++k) y[i * NOUT + k] = o[k];
}

hipError_t launch_mlp_infer(const uint16_t *wbf, const float *feat, uint64_t n, float *y, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_mlp_infer<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(wbf, feat, n, y);
    return hipGetLastError();
}

// fp32 master weights -> bf16 copy
__global__ void k_to_bf16(const float *__restrict__ w, uint16_t *__restrict__ wbf) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < NPARAM) wbf[k] = f2bf(w[k]);
}

hipError_t launch_to_bf16(const float *w, uint16_t *wbf, hipStream_t s) {
    k_to_bf16<<<(NPARAM + 255) / 256, 256, 0, s>>>(w, wbf);
    return hipGetLastError();
}

// Gradient of the mean loss over samples [b0, b0 + nb) with respect to the weights (the
// forward pass uses the bf16 copy, gradients are fp32).  Loss of a sample: squared error of
// y[0] against cost, plus the softmax cross-entropy of logits y[1..2] against bucket.
// One thread per sample; per-block sums in LDS, one atomic per parameter and block.
__global__ __launch_bounds__(256) void k_mlp_grad(const uint16_t *__restrict__ wbf, const float *__restrict__ feat,
                                                  const float *__restrict__ cost, const uint8_t *__restrict__ bucket,
                                                  uint64_t b0, uint32_t nb, float *__restrict__ grad,
                                                  float *__restrict__ loss) {
    __shared__ uint16_t w[NPARAM];
    __shared__ float g[NPARAM];
    for (int k = threadIdx.x; k < NPARAM; k += blockDim.x) {
        w[k] = wbf[k];
        g[k] = 0.0f;
    }
    __syncthreads();
    const uint32_t j0 = blockIdx.x * blockDim.x + threadIdx.x;
    float my_loss = 0.0f;
    if (j0 < nb) {
        const uint64_t i = b0 + j0;
        const float inv = 1.0f / (float)nb;
        float x[NFEAT], h1[NHID], h2[NHID], y[NOUT];
        for (int k = 0; k < NFEAT; ++k) x[k] = feat[i * NFEAT + k];
        mlp_forward(w, x, h1, h2, y);
        // output gradients
        float dy[NOUT];
        const float e = y[0] - cost[i];
        dy[0] = 2.0f * e * inv;
        const float m = fmaxf(y[1], y[2]);
        const float e1 = expf(y[1] - m), e2 = expf(y[2] - m);
        const float p1 = e1 / (e1 + e2), p2 = e2 / (e1 + e2);
        const int t = bucket[i] ? 1 : 0;
        dy[1] = (p1 - (t == 0 ? 1.0f : 0.0f)) * inv;
        dy[2] = (p2 - (t == 1 ? 1.0f : 0.0f)) * inv;
        my_loss = e * e - logf(t == 0 ? fmaxf(p1, 1e-30f) : fmaxf(p2, 1e-30f));
        // layer 3
        float dh2[NHID];
        for (int k = 0; k < NHID; ++k) {
            float acc = 0.0f;
            for (int o = 0; o < NOUT; ++o) {
                atomicAdd(&g[OW3 + k * NOUT + o], h2[k] * dy[o]);
                acc += bf2f(w[OW3 + k * NOUT + o]) * dy[o];
            }
            dh2[k] = h2[k] > 0.0f ? acc : 0.0f;
        }
        for (int o = 0; o < NOUT; ++o) atomicAdd(&g[OB3 + o], dy[o]);
        // layer 2
        float dh1[NHID];
        for (int k = 0; k < NHID; ++k) dh1[k] = 0.0f;
        for (int j = 0; j < NHID; ++j) {
            const float d = dh2[j];
            if (d == 0.0f) continue;
            atomicAdd(&g[OB2 + j], d);
            for (int k = 0; k < NHID; ++k) {
                atomicAdd(&g[OW2 + k * NHID + j], h1[k] * d);
                dh1[k] += bf2f(w[OW2 + k * NHID + j]) * d;
            }
        }
        // layer 1
        for (int j = 0; j < NHID; ++j) {
            const float d = h1[j] > 0.0f ? dh1[j] : 0.0f;
            if (d == 0.0f) continue;
            atomicAdd(&g[OB1 + j], d);
            for (int k = 0; k < NFEAT; ++k) atomicAdd(&g[OW1 + k * NHID + j], x[k] * d);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NPARAM; k += blockDim.x)
        if (g[k] != 0.0f) atomicAdd(&grad[k], g[k]);
    // loss sum (for the gradient check; training passes no loss buffer)
    float s = my_loss;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (loss && (threadIdx.x & 63) == 0) atomicAdd(loss, s);
}

hipError_t launch_mlp_grad(const uint16_t *wbf, const float *feat, const float *cost, const uint8_t *bucket,
                           uint64_t b0, uint32_t nb, float *grad, float *loss, hipStream_t s) {
    if (nb == 0) return hipSuccess;
    k_mlp_grad<<<(nb + 255) / 256, 256, 0, s>>>(wbf, feat, cost, bucket, b0, nb, grad, loss);
    return hipGetLastError();
}

// Adam step (step number t >= 1) on the fp32 master weights; clears the gradient and
// refreshes the bf16 copy
__global__ void k_adam(float *__restrict__ w, float *__restrict__ grad, float *__restrict__ m1,
                       float *__restrict__ m2, uint16_t *__restrict__ wbf, float lr, int t) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NPARAM) return;
    const float b1 = 0.9f, b2 = 0.999f;
    const float gk = grad[k];
    m1[k] = b1 * m1[k] + (1.0f - b1) * gk;
    m2[k] = b2 * m2[k] + (1.0f - b2) * gk * gk;
    const float mh = m1[k] / (1.0f - powf(b1, (float)t)), vh = m2[k] / (1.0f - powf(b2, (float)t));
    w[k] -= lr * mh / (sqrtf(vh) + 1e-8f);
    grad[k] = 0.0f;
    wbf[k] = f2bf(w[k]);
}

hipError_t launch_adam(float *w, float *grad, float *m1, float *m2, uint16_t *wbf, float lr, int t, hipStream_t s) {
    k_adam<<<(NPARAM + 255) / 256, 256, 0, s>>>(w, grad, m1, m2, wbf, lr, t);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scheduler hooks

// level key of each curve-ordered record for the learned order: 2 level + (predicted cost
// above the threshold), so that within each level the costly half comes last; the walk
// bucket of each record (1: start at the anchor)
__global__ void k_learned_keys(const float *__restrict__ y, const uint8_t *__restrict__ level, uint64_t n,
                               uint64_t base, float thr, unsigned long long *__restrict__ keys,
                               uint32_t *__restrict__ vals, uint8_t *__restrict__ wbucket) {
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = 2ull * level[i] + (y[i * NOUT] > thr ? 1ull : 0ull);
    vals[i] = (uint32_t)(base + i);
    wbucket[i] = y[i * NOUT + 2] > y[i * NOUT + 1] ? 1 : 0;
}

hipError_t launch_learned_keys(const float *y, const uint8_t *level, uint64_t n, uint64_t base, float thr,
                               unsigned long long *keys, uint32_t *vals, uint8_t *wbucket, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_learned_keys<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(y, level, n, base, thr, keys, vals, wbucket);
    return hipGetLastError();
}

// training labels of the records of a finished plain run: log2(1 + attempts), and bucket 1
// when the anchor is closer to the point than each record within 4 places on the curve that
// belongs to a lower BRIO level (the neighbours that are sure to be inserted before the
// point, hence walk starts the default rule may take); 0 when there is no such record
__global__ void k_labels(const Vert *__restrict__ V, uint64_t base, uint64_t n, const Cloud *__restrict__ clouds,
                         const uint32_t *__restrict__ anchor, const uint8_t *__restrict__ level,
                         const uint32_t *__restrict__ attempts, float *__restrict__ cost,
                         uint8_t *__restrict__ bucket) {
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = (uint32_t)(base + i);
    const Vert a = V[p];
    const Cloud cl = clouds[a.idx >> 32];
    cost[i] = log2f(1.0f + (float)attempts[i]);
    const uint32_t q = anchor[i];
    uint8_t b = 0;
    if (q != NONE) {
        float dn = 1e30f;
        for (uint32_t d = 1; d <= 4; ++d) {
            if (p + d < cl.hi && level[i + d] < level[i]) dn = fminf(dn, ldist(a, V, p + d, true, 1.0));
            if (p >= cl.lo + d && level[i - d] < level[i]) dn = fminf(dn, ldist(a, V, p - d, true, 1.0));
        }
        b = dn < 1e30f && ldist(a, V, q, true, 1.0) < dn ? 1 : 0;
    }
    bucket[i] = b;
}

hipError_t launch_labels(const Vert *V, uint64_t base, uint64_t n, const Cloud *clouds, const uint32_t *anchor,
                         const uint8_t *level, const uint32_t *attempts, float *cost, uint8_t *bucket,
                         hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_labels<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(V, base, n, clouds, anchor, level, attempts, cost, bucket);
    return hipGetLastError();
}

}  // namespace dtk

// Training kernels of the learned step schedule (forward, backward and Adam
// for the 12 -> 64 -> 64 -> 9 network of mlp_dev.h), and batched inference
// for tests.
//
// k_mlp_grad: one wave per workgroup; each wave takes a contiguous slice of
// a (shuffled) mini-batch, runs forward and backward per sample with lane j
// owning hidden unit j, accumulates its parameters' gradients in registers
// and writes one partial gradient vector. k_mlp_adam sums the partials in a
// fixed order (deterministic) and applies Adam. The transposed access to W2
// in the backward pass (column j of W2 for the layer-1 gradient) reads a
// copy of W2 in LDS, which lanes read at consecutive addresses.
#include "mlp_dev.h"

namespace ppsp {

__global__ __launch_bounds__(MLP_H) void k_mlp_forward(const float *P, const float *X, uint32_t n, float *logits) {
    MlpLane L;
    mlp_load_lane(P, L);
    for (uint32_t s = blockIdx.x; s < n; s += gridDim.x) {
        float x[MLP_F];
#pragma unroll
        for (int i = 0; i < MLP_F; i++) x[i] = X[(uint64_t)s * MLP_F + i];
        float z1, h1, z2, h2, lg[MLP_O];
        mlp_forward(L, x, z1, h1, z2, h2, lg);
        if (__lane_id() < (uint32_t)MLP_O) {
            float v = lg[0];
#pragma unroll
            for (int b = 1; b < MLP_O; b++) if (__lane_id() == (uint32_t)b) v = lg[b];
            logits[(uint64_t)s * MLP_O + __lane_id()] = v;
        }
    }
}

// Gradient of scale * sum of the row losses (mlp_dev.h) over samples
// idx[beg + w*per .. beg + (w+1)*per) (clipped to end) for wave w.
__global__ __launch_bounds__(MLP_H) void k_mlp_grad(const float *P, const float *X, const uint32_t *Y,
                                                    const uint32_t *idx, uint32_t beg, uint32_t end, uint32_t per,
                                                    float scale, float *partial, double *loss) {
    __shared__ float w2s[MLP_H * MLP_H];
    const uint32_t j = __lane_id();
    for (int k = 0; k < MLP_H; k++) w2s[k * MLP_H + j] = P[MLP_W2 + k * MLP_H + j];
    __syncthreads();
    MlpLane L;
    mlp_load_lane(P, L);
    float g1[MLP_F], gb1 = 0.f, g2[MLP_H], gb2 = 0.f, g3[MLP_O], gb3[MLP_O];
#pragma unroll
    for (int i = 0; i < MLP_F; i++) g1[i] = 0.f;
#pragma unroll
    for (int k = 0; k < MLP_H; k++) g2[k] = 0.f;
#pragma unroll
    for (int b = 0; b < MLP_O; b++) { g3[b] = 0.f; gb3[b] = 0.f; }
    double lsum = 0.0;
    const uint64_t s0 = (uint64_t)beg + (uint64_t)blockIdx.x * per;
    const uint64_t s1 = s0 + per < end ? s0 + per : end;
    for (uint64_t q = s0; q < s1; q++) {
        const uint32_t s = idx ? idx[q] : (uint32_t)q;
        float x[MLP_F];
#pragma unroll
        for (int i = 0; i < MLP_F; i++) x[i] = X[(uint64_t)s * MLP_F + i];
        const uint32_t yy = Y[s];
        const uint32_t y = yy % MLP_K, m = yy / MLP_K;   // bin label, mode label (0: none, 1 sparse, 2 dense)
        float z1, h1, z2, h2, lg[MLP_O];
        mlp_forward(L, x, z1, h1, z2, h2, lg);
        // softmax cross-entropy
        float mx = lg[0];
#pragma unroll
        for (int b = 1; b < MLP_K; b++) mx = fmaxf(mx, lg[b]);
        float den = 0.f, ly = 0.f;
#pragma unroll
        for (int b = 0; b < MLP_K; b++) {
            den += expf(lg[b] - mx);
            if ((uint32_t)b == y) ly = lg[b];
        }
        lsum += (double)(logf(den) + mx - ly);
        float dl[MLP_O];
#pragma unroll
        for (int b = 0; b < MLP_K; b++) dl[b] = scale * (expf(lg[b] - mx) / den - ((uint32_t)b == y ? 1.f : 0.f));
        dl[MLP_K] = 0.f;
        if (m) {
            // logistic loss of the mode logit z against t = (m == 2):
            // log(1 + e^z) - t z, computed without overflow; its derivative is sigmoid(z) - t
            const float z = lg[MLP_K], t = m == 2 ? 1.f : 0.f;
            lsum += (double)(fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - t * z);
            dl[MLP_K] = scale * (1.f / (1.f + expf(-z)) - t);
        }
        // layer 3
        float dh2 = 0.f;
#pragma unroll
        for (int b = 0; b < MLP_O; b++) {
            g3[b] = fmaf(dl[b], h2, g3[b]);
            gb3[b] += dl[b];
            dh2 = fmaf(L.w3[b], dl[b], dh2);
        }
        const float dz2 = z2 > 0.f ? dh2 : 0.f;
        // layer 2: dW2[j][k] = dz2_j * h1_k; dh1_j = sum_m W2[m][j] * dz2_m
        float dh1 = 0.f;
#pragma unroll
        for (int k = 0; k < MLP_H; k++) {
            g2[k] = fmaf(dz2, __shfl(h1, k), g2[k]);
            dh1 = fmaf(w2s[k * MLP_H + j], __shfl(dz2, k), dh1);
        }
        gb2 += dz2;
        const float dz1 = z1 > 0.f ? dh1 : 0.f;
#pragma unroll
        for (int i = 0; i < MLP_F; i++) g1[i] = fmaf(dz1, x[i], g1[i]);
        gb1 += dz1;
    }
    float *out = partial + (uint64_t)blockIdx.x * MLP_NPARAM;
#pragma unroll
    for (int i = 0; i < MLP_F; i++) out[MLP_W1 + j * MLP_F + i] = g1[i];
    out[MLP_B1 + j] = gb1;
#pragma unroll
    for (int k = 0; k < MLP_H; k++) out[MLP_W2 + j * MLP_H + k] = g2[k];
    out[MLP_B2 + j] = gb2;
#pragma unroll
    for (int b = 0; b < MLP_O; b++) out[MLP_W3 + b * MLP_H + j] = g3[b];
    if (j < (uint32_t)MLP_O) {
        float v = gb3[0];
#pragma unroll
        for (int b = 1; b < MLP_O; b++) if (j == (uint32_t)b) v = gb3[b];
        out[MLP_B3 + j] = v;
    }
    if (j == 0) loss[blockIdx.x] = lsum;
}

// Sum of nw partial gradients per parameter, in wave order.
__device__ __forceinline__ float sum_partials(const float *partial, uint32_t nw, uint32_t p) {
    float g = 0.f;
    for (uint32_t w = 0; w < nw; w++) g += partial[(uint64_t)w * MLP_NPARAM + p];
    return g;
}

__global__ void k_mlp_reduce(const float *partial, uint32_t nw, float *grad) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < (uint32_t)MLP_NPARAM) grad[p] = sum_partials(partial, nw, p);
}

// Adam (Kingma and Ba) with bias correction; step t >= 1.
__global__ void k_mlp_adam(float *P, float *m, float *v, const float *partial, uint32_t nw, float lr, float b1,
                           float b2, float eps, uint32_t t) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (uint32_t)MLP_NPARAM) return;
    const float g = sum_partials(partial, nw, p);
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.f - powf(b1, (float)t));
    const float vh = vv / (1.f - powf(b2, (float)t));
    P[p] -= lr * mh / (sqrtf(vh) + eps);
}

hipError_t launch_mlp_forward(const float *P, const float *X, uint32_t n, float *logits, hipStream_t st) {
    const uint32_t grid = n < 4096 ? (n ? n : 1) : 4096;
    k_mlp_forward<<<grid, MLP_H, 0, st>>>(P, X, n, logits);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *P, const float *X, const uint32_t *Y, const uint32_t *idx, uint32_t beg,
                           uint32_t end, uint32_t per, uint32_t nw, float scale, float *partial, double *loss,
                           hipStream_t st) {
    k_mlp_grad<<<nw, MLP_H, 0, st>>>(P, X, Y, idx, beg, end, per, scale, partial, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(const float *partial, uint32_t nw, float *grad, hipStream_t st) {
    k_mlp_reduce<<<(MLP_NPARAM + 255) / 256, 256, 0, st>>>(partial, nw, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *P, float *m, float *v, const float *partial, uint32_t nw, float lr, uint32_t t,
                           hipStream_t st) {
    k_mlp_adam<<<(MLP_NPARAM + 255) / 256, 256, 0, st>>>(P, m, v, partial, nw, lr, 0.9f, 0.999f, 1e-8f, t);
    return hipGetLastError();
}

}  // namespace ppsp

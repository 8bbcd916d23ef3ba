// The learned step schedule: a 12 -> 64 -> 64 -> 9 multilayer perceptron
// that picks, per search and round, the multiplier 2^(b-4) (b = 0..7) of the
// search's base Delta (logits 0..7) and whether its frontier becomes dense
// (logit 8 > 0; the dense mode of Appendix B). It only chooses thresholds and
// the frontier's container, and any threshold sequence gives exact distances
// (Theorems bids-correctness and bdastar-correctness hold for every stepping
// rule), so it changes speed, never results.
//
// Parameters, one flat float array (row-major):
//     W1 [64][12]   b1 [64]   W2 [64][64]   b2 [64]   W3 [9][64]   b3 [9]
// Activations: ReLU after both hidden layers. Training loss per row: softmax
// cross-entropy of the 8 bin logits against the best bin, plus, for rows with
// a mode label, the logistic loss of logit 8 against it. A label is
// y = bin + 8 * m, m = 0 (no mode label), 1 (sparse) or 2 (dense).
//
// Wave-parallel evaluation: lane j of a 64-lane wave owns hidden unit j of
// both layers (row j of W1 and W2, column j of W3), so a forward pass is 12 +
// 64 fused multiply-adds per lane, 64 lane reads for the layer-2 inputs and 9
// wave sums for the logits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppsp {

constexpr int MLP_F = 12;        // features
constexpr int MLP_H = 64;        // hidden units per layer (= wave size)
constexpr int MLP_K = 8;         // Delta-multiplier bins
constexpr int MLP_O = MLP_K + 1; // outputs: the bin logits and the dense-mode logit
constexpr int MLP_Y = 3 * MLP_K; // labels: bin + 8 * (0 no mode label | 1 sparse | 2 dense)
constexpr int MLP_W1 = 0;
constexpr int MLP_B1 = MLP_W1 + MLP_H * MLP_F;
constexpr int MLP_W2 = MLP_B1 + MLP_H;
constexpr int MLP_B2 = MLP_W2 + MLP_H * MLP_H;
constexpr int MLP_W3 = MLP_B2 + MLP_H;
constexpr int MLP_B3 = MLP_W3 + MLP_O * MLP_H;
constexpr int MLP_NPARAM = MLP_B3 + MLP_O;   // 5577

// One lane's share of the parameters (hidden unit j = lane).
struct MlpLane {
    float w1[MLP_F];
    float b1;
    float w2[MLP_H];
    float b2;
    float w3[MLP_O];   // column j of W3
    float b3[MLP_O];   // the same on every lane
};

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <typename T>
__device__ __forceinline__ float param_at(const T *p, uint32_t k);
template <>
__device__ __forceinline__ float param_at<float>(const float *p, uint32_t k) { return p[k]; }
template <>
__device__ __forceinline__ float param_at<uint16_t>(const uint16_t *p, uint32_t k) { return bf16_to_f32(p[k]); }

template <typename T>
__device__ __forceinline__ void mlp_load_lane(const T *P, MlpLane &L) {
    const uint32_t j = __lane_id();
#pragma unroll
    for (int i = 0; i < MLP_F; i++) L.w1[i] = param_at(P, MLP_W1 + j * MLP_F + i);
    L.b1 = param_at(P, MLP_B1 + j);
#pragma unroll
    for (int k = 0; k < MLP_H; k++) L.w2[k] = param_at(P, MLP_W2 + j * MLP_H + k);
    L.b2 = param_at(P, MLP_B2 + j);
#pragma unroll
    for (int b = 0; b < MLP_O; b++) {
        L.w3[b] = param_at(P, MLP_W3 + b * MLP_H + j);
        L.b3[b] = param_at(P, MLP_B3 + b);
    }
}

__device__ __forceinline__ float wave_sum_f32(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Forward pass of one sample x (the same on every lane). Returns this lane's
// pre-activations z1, z2 and the MLP_O logits (the same on every lane).
__device__ __forceinline__ void mlp_forward(const MlpLane &L, const float *x, float &z1, float &h1, float &z2,
                                            float &h2, float *logit) {
    float a = L.b1;
#pragma unroll
    for (int i = 0; i < MLP_F; i++) a = fmaf(L.w1[i], x[i], a);
    z1 = a;
    h1 = fmaxf(a, 0.f);
    float c = L.b2;
#pragma unroll
    for (int k = 0; k < MLP_H; k++) c = fmaf(L.w2[k], __shfl(h1, k), c);
    z2 = c;
    h2 = fmaxf(c, 0.f);
#pragma unroll
    for (int b = 0; b < MLP_O; b++) logit[b] = L.b3[b] + wave_sum_f32(L.w3[b] * h2);
}

// Index of the largest bin logit (the lowest index among equal ones).
__device__ __forceinline__ uint32_t mlp_argmax(const float *logit) {
    uint32_t best = 0;
#pragma unroll
    for (int b = 1; b < MLP_K; b++)
        if (logit[b] > logit[best]) best = b;
    return best;
}

}  // namespace ppsp

// Learned proposal correction: features and forward pass of the 3-layer
// MLP, shared by the sampler (inference at every site) and the training
// kernels.  Parameter vector layout (float32, row major [out][in]):
//   W1 [64][64] | b1 [64] | W2 [64][64] | b2 [64] | W3 [64] | b3 [1]
#pragma once

#include "device.hpp"

namespace tnmc {

constexpr int MLP_IN = 64, MLP_H = 64;
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = 4096, MLP_OFF_W2 = 4160, MLP_OFF_B2 = 8256;
constexpr int MLP_OFF_W3 = 8320, MLP_OFF_B3 = 8384, MLP_NPARAM = 8385;

// Learned correction (optional) of a sampling launch: the parameter vector
// above and the horizontal couplings for the features.
struct MlpArgs {
    const float *params;
    const float *Jh;
};

// Features of site (r, c): 20 horizontal couplings (rows r-2..r+2, columns
// c-2..c+1), 20 vertical couplings (rows r-2..r+1, columns c-2..c+2), the
// 12 already-sampled spins of the 5x5 window (rows r-2, r-1 at c-2..c+2 and
// row r at c-2, c-1), the low-chi logit clipped to [-30, 30] / 8; zero
// outside the lattice and in slots 53..63.  spin(rr, cc) returns -1 / +1.
template <typename SpinFn>
__device__ __forceinline__ void mlp_features(const float *jh, const float *jv, int L, int r, int c,
                                             SpinFn spin, float logit, float *x) {
#pragma unroll
    for (int k = 0; k < MLP_IN; ++k) x[k] = 0.f;
#pragma unroll
    for (int dr = -2; dr <= 2; ++dr)
#pragma unroll
        for (int dc = -2; dc <= 1; ++dc) {
            const int rr = r + dr, cc = c + dc;
            if (rr >= 0 && rr < L && cc >= 0 && cc < L - 1) x[(dr + 2) * 4 + (dc + 2)] = jh[(size_t)rr * (L - 1) + cc];
        }
#pragma unroll
    for (int dr = -2; dr <= 1; ++dr)
#pragma unroll
        for (int dc = -2; dc <= 2; ++dc) {
            const int rr = r + dr, cc = c + dc;
            if (rr >= 0 && rr < L - 1 && cc >= 0 && cc < L) x[20 + (dr + 2) * 5 + (dc + 2)] = jv[(size_t)rr * L + cc];
        }
#pragma unroll
    for (int dr = -2; dr <= -1; ++dr)
#pragma unroll
        for (int dc = -2; dc <= 2; ++dc) {
            const int rr = r + dr, cc = c + dc;
            if (rr >= 0 && cc >= 0 && cc < L) x[40 + (dr + 2) * 5 + (dc + 2)] = spin(rr, cc);
        }
#pragma unroll
    for (int dc = -2; dc <= -1; ++dc) {
        const int cc = c + dc;
        if (cc >= 0) x[50 + dc + 2] = spin(r, cc);
    }
    x[52] = fminf(fmaxf(logit, -30.f), 30.f) * 0.125f;
}

// d = W3 . tanh(W2 tanh(W1 x + b1) + b2) + b3 with the parameters in P
// (shared or global memory); float32 accumulation.
__device__ __forceinline__ float mlp_forward(const float *P, const float *x) {
    float h1[MLP_H];
#pragma unroll
    for (int o = 0; o < MLP_H; ++o) {
        float a = P[MLP_OFF_B1 + o];
        const float *w = P + MLP_OFF_W1 + o * MLP_IN;
#pragma unroll
        for (int i = 0; i < MLP_IN; ++i) a += w[i] * x[i];
        h1[o] = tanhf(a);
    }
    float d = P[MLP_OFF_B3];
#pragma unroll
    for (int o = 0; o < MLP_H; ++o) {
        float a = P[MLP_OFF_B2 + o];
        const float *w = P + MLP_OFF_W2 + o * MLP_H;
#pragma unroll
        for (int i = 0; i < MLP_H; ++i) a += w[i] * h1[i];
        d += P[MLP_OFF_W3 + o] * tanhf(a);
    }
    return d;
}

}  // namespace tnmc

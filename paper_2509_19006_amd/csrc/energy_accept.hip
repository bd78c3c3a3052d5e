// Exact energies (Eq. (1)) and the Metropolis independence step (Eq. (10)).
// This file is compiled with -ffp-contract=off: the accept log-ratio is
// rounded once per operation, as its definition states.
#include "device.hpp"

#pragma clang fp contract(off)

namespace tnmc {

// One wave per (sample, instance).  Each lane takes whole rows: the
// horizontal bonds of row r and the vertical bonds from row r to r+1.  With
// +-1 or 2^-20-grid couplings every partial sum is exact in float64, so the
// result does not depend on the summation order.
__global__ void __launch_bounds__(64)
k_energy(const InstDesc *__restrict__ desc, int n_samples, const uint64_t *__restrict__ spins,
         const float *__restrict__ Jh_all, const float *__restrict__ Jv_all, double *__restrict__ E_out) {
    const int inst = blockIdx.y, n = blockIdx.x, lane = threadIdx.x;
    const InstDesc d = desc[inst];
    const int L = d.L, W = d.W;
    const uint64_t *s = spins + (size_t)n_samples * d.word_prefix + (size_t)n * L * W;
    const float *jh = Jh_all + d.off_h, *jv = Jv_all + d.off_v;
    double e = 0.0;
    for (int r = lane; r < L; r += 64) {
        const uint64_t *row = s + (size_t)r * W, *nxt = s + (size_t)(r + 1) * W;
        for (int c = 0; c < L; ++c) {
            const double sc = ((row[c >> 6] >> (c & 63)) & 1) ? 1.0 : -1.0;
            if (c + 1 < L) {
                const double sr = ((row[(c + 1) >> 6] >> ((c + 1) & 63)) & 1) ? 1.0 : -1.0;
                e -= (double)jh[(size_t)r * (L - 1) + c] * (sc * sr);
            }
            if (r + 1 < L) {
                const double sd = ((nxt[c >> 6] >> (c & 63)) & 1) ? 1.0 : -1.0;
                e -= (double)jv[(size_t)r * L + c] * (sc * sd);
            }
        }
    }
    for (int m = 32; m > 0; m >>= 1) e += __shfl_xor(e, m, 64);
    if (lane == 0) E_out[(size_t)inst * n_samples + n] = e;
}

struct Chain {
    double cur_logq, cur_E;
    int64_t cur_index, n_acc, n_trials, initialised;
};

// One thread per instance walks its proposals in order.
__global__ void k_accept(int B, int n, const double *__restrict__ logq, const double *__restrict__ E,
                         const double *__restrict__ beta, Chain *__restrict__ chain, uint64_t seed,
                         uint64_t step_offset, uint8_t *__restrict__ acc, int64_t *__restrict__ state) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    Chain ch = chain[i];
    const double b = beta[i];
    for (int k = 0; k < n; ++k) {
        const uint64_t g = step_offset + (uint64_t)k;
        const double lq = logq[(size_t)i * n + k], e = E[(size_t)i * n + k];
        uint8_t a = 0;
        if (!ch.initialised) {
            ch.initialised = 1;
            ch.cur_logq = lq; ch.cur_E = e; ch.cur_index = (int64_t)g;
            a = 1;
        } else {
            const double d_logq = ch.cur_logq - lq;
            const double d_E = ch.cur_E - e;
            const double prod = b * d_E;
            const double delta = d_logq + prod;
            const double u = philox_unit(seed, (uint32_t)g, 0u, (uint32_t)i, 1u);
            const bool ok = (delta >= 0.0) || (u < exp(delta));
            ch.n_trials += 1;
            if (ok) {
                ch.n_acc += 1;
                ch.cur_logq = lq; ch.cur_E = e; ch.cur_index = (int64_t)g;
                a = 1;
            }
        }
        acc[(size_t)i * n + k] = a;
        if (state) state[(size_t)i * n + k] = ch.cur_index;
    }
    chain[i] = ch;
}

__global__ void k_philox(uint64_t seed, const uint32_t *__restrict__ c0, uint32_t c1, uint32_t c2,
                         uint32_t c3, int n, double *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = philox_unit(seed, c0[k], c1, c2, c3);
}

hipError_t launch_energy(const InstDesc *desc, int B, int n_samples, const uint64_t *spins,
                         const float *Jh, const float *Jv, double *E, hipStream_t st) {
    hipLaunchKernelGGL(k_energy, dim3(n_samples, B), dim3(64), 0, st, desc, n_samples, spins, Jh, Jv, E);
    return hipGetLastError();
}

hipError_t launch_accept(int B, int n, const double *logq, const double *E, const double *beta,
                         void *chain, uint64_t seed, uint64_t off, uint8_t *acc, int64_t *state,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_accept, dim3((B + 63) / 64), dim3(64), 0, st, B, n, logq, E, beta,
                       reinterpret_cast<Chain *>(chain), seed, off, acc, state);
    return hipGetLastError();
}

hipError_t launch_philox(uint64_t seed, const uint32_t *c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         int n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_philox, dim3((n + 255) / 256), dim3(256), 0, st, seed, c0, c1, c2, c3, n, out);
    return hipGetLastError();
}

}  // namespace tnmc

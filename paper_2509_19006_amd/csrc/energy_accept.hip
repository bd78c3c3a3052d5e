// Exact energies (Eq. (1)) and the Metropolis independence step (Eq. (10)).
// This file is compiled with -ffp-contract=off and the accept function
// switches contraction off itself: the log-ratio is rounded once per
// operation, as its definition states.
#include "energy_accept_device.hpp"

#pragma clang fp contract(off)

namespace tnmc {

// One wave per (sample, instance).
__global__ void __launch_bounds__(64)
k_energy(const InstDesc *__restrict__ desc, int n_samples, const uint64_t *__restrict__ spins,
         const float *__restrict__ Jh_all, const float *__restrict__ Jv_all, double *__restrict__ E_out) {
    const int inst = blockIdx.y, n = blockIdx.x, lane = threadIdx.x;
    const InstDesc d = desc[inst];
    const uint64_t *s = spins + (size_t)n_samples * d.word_prefix + (size_t)n * d.L * d.W;
    const double e = energy_wave(d, s, Jh_all, Jv_all, lane);
    if (lane == 0) E_out[(size_t)inst * n_samples + n] = e;
}

// One thread per instance walks its proposals in order.
__global__ void k_accept(int B, int n, const double *__restrict__ logq, const double *__restrict__ E,
                         const double *__restrict__ beta, Chain *__restrict__ chain, uint64_t seed,
                         uint64_t step_offset, uint8_t *__restrict__ acc, int64_t *__restrict__ state) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    accept_chain(i, n, logq + (size_t)i * n, E + (size_t)i * n, beta[i], chain + i, seed, step_offset,
                 acc + (size_t)i * n, state ? state + (size_t)i * n : nullptr);
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

// Exact energies (Eq. (1)) and the Metropolis independence step (Eq. (10)).
// This file is compiled with -ffp-contract=off and the accept function
// switches contraction off itself: the log-ratio is rounded once per
// operation, as its definition states.
#include "energy_accept_device.hpp"

#pragma clang fp contract(off)

namespace tnmc {

// Energies of a run of instances that share the side L (one wave per
// (sample, instance of the run)); instance j of the run has its couplings
// at Jh + j*stride_h, Jv + j*stride_v and its configurations at
// spins + j*inst_words.  With E_int non-NULL the energy is also summed in
// int32 from the couplings taken as integers; an instance with a coupling
// that is not an integer gets INT32_MIN there.
__global__ void __launch_bounds__(64)
k_energy_run(int L, int n_samples, const uint64_t *__restrict__ spins, int64_t inst_words,
             const float *__restrict__ Jh, int64_t stride_h, const float *__restrict__ Jv, int64_t stride_v,
             double *__restrict__ E_out, int32_t *__restrict__ E_int) {
    const int j = blockIdx.y, n = blockIdx.x, lane = threadIdx.x;
    InstDesc d{};
    d.L = L;
    d.W = (L + 63) / 64;
    d.off_h = (int64_t)j * stride_h;
    d.off_v = (int64_t)j * stride_v;
    const uint64_t *s = spins + (size_t)j * inst_words + (size_t)n * L * d.W;
    int64_t ei = 0;
    const double e = energy_wave(d, s, Jh, Jv, lane, E_int ? &ei : nullptr);
    if (lane == 0) {
        E_out[(size_t)j * n_samples + n] = e;
        if (E_int) E_int[(size_t)j * n_samples + n] = ei == INT64_MIN ? INT32_MIN : (int32_t)ei;
    }
}

// Replica overlap of two Markov chains of the same instances: for each
// (step k, instance j of a run of equal L), q = (1/L^2) sum_i s_i^a s_i^b of
// the two chains' current states, read from this call's proposals by their
// global indices (state - offset); a state from before this call gives NaN.
// One wave per (step, instance); popcount of the XOR of the packed rows.
__global__ void __launch_bounds__(64)
k_overlap_run(int L, int n_samples, const uint64_t *__restrict__ sa, const int64_t *__restrict__ ia,
              const uint64_t *__restrict__ sb, const int64_t *__restrict__ ib, int64_t inst_words,
              int64_t offset, double *__restrict__ q_out) {
    const int j = blockIdx.y, k = blockIdx.x, lane = threadIdx.x;
    const int W = (L + 63) / 64;
    const int64_t xa = ia[(size_t)j * n_samples + k] - offset, xb = ib[(size_t)j * n_samples + k] - offset;
    double *q = q_out + (size_t)j * n_samples + k;
    if (xa < 0 || xa >= n_samples || xb < 0 || xb >= n_samples) {
        if (lane == 0) *q = __builtin_nan("");
        return;
    }
    const uint64_t *a = sa + (size_t)j * inst_words + (size_t)xa * L * W;
    const uint64_t *b = sb + (size_t)j * inst_words + (size_t)xb * L * W;
    const uint64_t tail = (L & 63) ? ((uint64_t(1) << (L & 63)) - 1) : ~uint64_t(0);
    int64_t diff = 0;
    for (int w = lane; w < L * W; w += 64) {
        uint64_t x = a[w] ^ b[w];
        if ((w % W) == W - 1) x &= tail;
        diff += __popcll(x);
    }
    for (int m = 32; m > 0; m >>= 1) diff += __shfl_xor(diff, m, 64);
    if (lane == 0) *q = 1.0 - 2.0 * (double)diff / ((double)L * (double)L);
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

hipError_t launch_energy_run(int L, int n_inst, int n_samples, const uint64_t *spins, int64_t inst_words,
                             const float *Jh, int64_t stride_h, const float *Jv, int64_t stride_v, double *E,
                             int32_t *E_int, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_run, dim3(n_samples, n_inst), dim3(64), 0, st, L, n_samples, spins, inst_words, Jh,
                       stride_h, Jv, stride_v, E, E_int);
    return hipGetLastError();
}

hipError_t launch_overlap_run(int L, int n_inst, int n_samples, const uint64_t *sa, const int64_t *ia,
                              const uint64_t *sb, const int64_t *ib, int64_t inst_words, int64_t offset,
                              double *q, hipStream_t st) {
    hipLaunchKernelGGL(k_overlap_run, dim3(n_samples, n_inst), dim3(64), 0, st, L, n_samples, sa, ia, sb, ib,
                       inst_words, offset, q);
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
